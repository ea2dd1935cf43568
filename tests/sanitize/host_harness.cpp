// Host-side harness of libugks for AddressSanitizer / UndefinedBehaviorSanitizer
// builds: drives input validation, mesh relabelling, geometry building, the
// push sweep's colouring and the footprint plan through the C ABI on small
// procedurally built meshes, with valid and invalid inputs.  On a machine
// without a GPU, ugks_create runs every host step and then fails at its
// first device allocation (UGKS_ERR_ALLOC or UGKS_ERR_HIP); with a GPU it
// succeeds and the handle is destroyed again.  Exit status 0 when every
// expectation holds.
#include "ugks.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

namespace {

int g_checks = 0, g_fail = 0;

void expect(bool ok, const std::string &what)
{
    ++g_checks;
    if (!ok) {
        ++g_fail;
        std::fprintf(stderr, "FAILED: %s\n", what.c_str());
    }
}

// A mesh held by value; view() gives the ABI struct pointing into it.
struct Mesh {
    int dim = 2, nc = 0;
    std::vector<double> vol, cen, nrm, area, fcen, shift;
    std::vector<int> fc, bc, bcid;
    ugks_mesh_t view() const
    {
        ugks_mesh_t m;
        std::memset(&m, 0, sizeof(m));
        m.dim = dim;
        m.n_cells = nc;
        m.n_faces = (int)area.size();
        m.cell_volume = vol.data();
        m.cell_centroid = cen.data();
        m.face_cells = fc.data();
        m.face_normal = nrm.data();
        m.face_area = area.data();
        m.face_centroid = fcen.data();
        m.face_shift = shift.empty() ? nullptr : shift.data();
        m.face_bc = bc.empty() ? nullptr : bc.data();
        m.face_bc_id = bcid.empty() ? nullptr : bcid.data();
        return m;
    }
    void face(int l, int r, const double *n, double a, const double *c, const double *s, int b, int id)
    {
        fc.push_back(l);
        fc.push_back(r);
        for (int d = 0; d < dim; ++d) {
            nrm.push_back(n[d]);
            fcen.push_back(c[d]);
            shift.push_back(s[d]);
        }
        area.push_back(a);
        bc.push_back(b);
        bcid.push_back(id);
    }
};

// nx x ny unit-square quadrilaterals; periodic in x; in y periodic too, or
// walls (bc id 0) below and above.
Mesh quad_mesh(int nx, int ny, bool walls)
{
    Mesh m;
    m.dim = 2;
    m.nc = nx * ny;
    const double hx = 1.0 / nx, hy = 1.0 / ny;
    auto id = [&](int i, int j) { return ((j + ny) % ny) * nx + (i + nx) % nx; };
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            m.vol.push_back(hx * hy);
            m.cen.push_back((i + 0.5) * hx);
            m.cen.push_back((j + 0.5) * hy);
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const double nxv[2] = {1.0, 0.0}, c[2] = {(i + 1) * hx, (j + 0.5) * hy};
            const double s[2] = {i == nx - 1 ? 1.0 : 0.0, 0.0};
            m.face(id(i, j), id(i + 1, j), nxv, hy, c, s, UGKS_BC_INTERIOR, 0);
        }
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const double up[2] = {0.0, 1.0}, down[2] = {0.0, -1.0}, c[2] = {(i + 0.5) * hx, j * hy};
            const double s0[2] = {0.0, 0.0};
            if (walls) {
                if (j == 0) m.face(id(i, 0), -1, down, hx, c, s0, UGKS_BC_WALL, 0);
                else if (j == ny) m.face(id(i, ny - 1), -1, up, hx, c, s0, UGKS_BC_WALL, 0);
                else m.face(id(i, j - 1), id(i, j), up, hx, c, s0, UGKS_BC_INTERIOR, 0);
            } else if (j < ny) {
                // the face below row j, from cell (i, j-1) to (i, j); for j = 0 the
                // left cell is the top row, the face sits at y = 1 in its frame and
                // the bottom row's image lies one period up
                const double cj[2] = {(i + 0.5) * hx, j == 0 ? 1.0 : j * hy};
                const double s[2] = {0.0, j == 0 ? 1.0 : 0.0};
                m.face(id(i, j - 1), id(i, j), up, hx, cj, s, UGKS_BC_INTERIOR, 0);
            }
        }
    return m;
}

// n^3 periodic unit-cube hexahedra.
Mesh hex_box(int n)
{
    Mesh m;
    m.dim = 3;
    m.nc = n * n * n;
    const double h = 1.0 / n;
    auto id = [&](int i, int j, int k) { return (((k + n) % n) * n + (j + n) % n) * n + (i + n) % n; };
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                m.vol.push_back(h * h * h);
                m.cen.push_back((i + 0.5) * h);
                m.cen.push_back((j + 0.5) * h);
                m.cen.push_back((k + 0.5) * h);
            }
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                for (int ax = 0; ax < 3; ++ax) {
                    int a[3] = {i, j, k}, b[3] = {i, j, k};
                    b[ax] += 1;
                    double nv[3] = {0, 0, 0}, c[3] = {(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h}, s[3] = {0, 0, 0};
                    nv[ax] = 1.0;
                    c[ax] = (a[ax] + 1) * h;
                    if (b[ax] == n) s[ax] = 1.0;
                    m.face(id(a[0], a[1], a[2]), id(b[0], b[1], b[2]), nv, h * h, c, s, UGKS_BC_INTERIOR, 0);
                }
    return m;
}

struct VGrid {
    int dim;
    std::vector<double> u, w;
    ugks_vgrid_t view() const { return ugks_vgrid_t{dim, (int)w.size(), u.data(), w.data()}; }
};

// n^dim trapezoid grid on [-L, L]^dim, or (scattered) the same points shifted
// off the lattice by a deterministic jitter so that no axis repeats.
VGrid vgrid(int dim, int n, double L, bool scattered)
{
    VGrid g;
    g.dim = dim;
    const double du = 2.0 * L / (n - 1);
    int total = 1;
    for (int d = 0; d < dim; ++d) total *= n;
    for (int k = 0; k < total; ++k) {
        int r = k;
        double w = 1.0;
        for (int d = 0; d < dim; ++d) {
            const int i = r % n;
            r /= n;
            double u = -L + i * du;
            if (scattered) u += 0.1 * du * std::sin(1.0 + 7.0 * k + 3.0 * d);
            g.u.push_back(u);
            w *= (i == 0 || i == n - 1) ? 0.5 * du : du;
        }
        g.w.push_back(w);
    }
    return g;
}

ugks_gas_t gas(int fstore, int mem, int sweep, const std::vector<double> &bc)
{
    ugks_gas_t g;
    std::memset(&g, 0, sizeof(g));
    g.Pr = 2.0 / 3.0;
    g.omega = 0.81;
    g.mu_ref = 0.05;
    g.cfl = 0.8;
    g.limiter_k = 1.0;
    g.limiter = 1;
    g.fstore = fstore;
    g.n_bc = bc.empty() ? 0 : 1;
    g.bc_prim = bc.empty() ? nullptr : bc.data();
    g.mem_mode = mem;
    g.sweep = sweep;
    return g;
}

std::vector<double> prim(const Mesh &m)
{
    std::vector<double> p;
    for (int i = 0; i < m.nc; ++i) {
        p.push_back(1.0 + 0.1 * std::sin(6.28 * m.cen[(size_t)i * m.dim]));
        for (int d = 0; d < m.dim; ++d) p.push_back(d == 0 ? 0.3 : 0.0);
        p.push_back(1.0);
    }
    return p;
}

// ugks_create on valid input: created (GPU present) or refused only at the
// first device allocation (no GPU).
void create_valid(const Mesh &m, const VGrid &v, const ugks_gas_t &g, const std::string &what)
{
    const ugks_mesh_t mv = m.view();
    const ugks_vgrid_t vv = v.view();
    const std::vector<double> p = prim(m);
    ugks_t *h = nullptr;
    const int rc = ugks_create(&mv, &vv, &g, p.data(), nullptr, &h);
    expect(rc == UGKS_OK || rc == UGKS_ERR_ALLOC || rc == UGKS_ERR_HIP,
           what + ": create returned " + std::to_string(rc) + " (" + ugks_last_error(nullptr) + ")");
    expect((rc == UGKS_OK) == (h != nullptr), what + ": handle set iff created");
    if (h) {
        expect(ugks_footprint_bytes(h) == ugks_footprint_estimate(&mv, &vv, &g), what + ": footprint");
        ugks_destroy(h);
    }
}

void create_invalid(const Mesh &m, const VGrid &v, const ugks_gas_t &g, const std::vector<double> &p,
                    const std::string &what)
{
    const ugks_mesh_t mv = m.view();
    const ugks_vgrid_t vv = v.view();
    ugks_t *h = reinterpret_cast<ugks_t *>(&g_checks);  // overwritten with NULL on failure
    const int rc = ugks_create(&mv, &vv, &g, p.data(), nullptr, &h);
    expect(rc == UGKS_ERR_ARG, what + ": expected UGKS_ERR_ARG, got " + std::to_string(rc));
    expect(h == nullptr, what + ": handle cleared");
    expect(std::strlen(ugks_last_error(nullptr)) > 0, what + ": message");
}

}  // namespace

int main()
{
    const std::vector<double> wall_bc = {1.0, 0.0, 0.0, 1.0};
    const Mesh per = quad_mesh(8, 6, false), chan = quad_mesh(7, 5, true), box = hex_box(4);
    const VGrid v2 = vgrid(2, 8, 4.0, false), v2s = vgrid(2, 7, 4.0, true), v3 = vgrid(3, 5, 4.0, false);

    // valid inputs: every storage, memory mode and sweep, tabulated and scattered velocities
    for (int fs : {UGKS_F64, UGKS_F32, UGKS_BF16})
        for (int mem : {UGKS_MEM_TWO_BUFFERS, UGKS_MEM_IN_PLACE})
            for (int sw : {UGKS_SWEEP_AUTO, UGKS_SWEEP_GATHER, UGKS_SWEEP_PUSH, UGKS_SWEEP_PUSH_UNORDERED}) {
                const std::string tag = "fs" + std::to_string(fs) + " mem" + std::to_string(mem) + " sweep" +
                                        std::to_string(sw);
                struct {
                    const Mesh *m;
                    const VGrid *v;
                    const std::vector<double> *bc;
                    const char *name;
                } cs[] = {{&per, &v2, nullptr, "periodic quads"},
                          {&chan, &v2s, &wall_bc, "channel, scattered velocities"},
                          {&box, &v3, nullptr, "periodic hexahedra"}};
                for (auto &c : cs) {
                    const ugks_gas_t g = gas(fs, mem, sw, c.bc ? *c.bc : std::vector<double>());
                    const ugks_mesh_t mv = c.m->view();
                    const ugks_vgrid_t vv = c.v->view();
                    const size_t est = ugks_footprint_estimate(&mv, &vv, &g);
                    expect(est > 0, std::string(c.name) + " " + tag + ": footprint");
                    create_valid(*c.m, *c.v, g, std::string(c.name) + " " + tag);
                }
            }

    // invalid inputs
    const ugks_gas_t g0 = gas(UGKS_F64, UGKS_MEM_TWO_BUFFERS, UGKS_SWEEP_AUTO, {});
    const std::vector<double> p0 = prim(per);
    {
        const ugks_mesh_t mv = per.view();
        const ugks_vgrid_t vv = v2.view();
        ugks_t *h = nullptr;
        expect(ugks_create(nullptr, &vv, &g0, p0.data(), nullptr, &h) == UGKS_ERR_ARG, "NULL mesh");
        expect(ugks_create(&mv, nullptr, &g0, p0.data(), nullptr, &h) == UGKS_ERR_ARG, "NULL velocity grid");
        expect(ugks_create(&mv, &vv, &g0, nullptr, nullptr, &h) == UGKS_ERR_ARG, "NULL initial state");
        expect(ugks_create(&mv, &vv, &g0, p0.data(), nullptr, nullptr) == UGKS_ERR_ARG, "NULL out");
        expect(ugks_footprint_estimate(nullptr, &vv, &g0) == 0, "footprint of NULL mesh");
    }
    auto bad_mesh = [&](const std::string &what, const std::function<void(Mesh &)> &edit) {
        Mesh m = per;
        edit(m);
        create_invalid(m, v2, g0, p0, what);
    };
    bad_mesh("dim 4", [](Mesh &m) { m.dim = 4; });
    bad_mesh("face cell out of range", [](Mesh &m) { m.fc[5] = m.nc; });
    bad_mesh("negative face cell", [](Mesh &m) { m.fc[4] = -3; });
    bad_mesh("interior face without a right cell", [](Mesh &m) { m.fc[3] = -1; });
    bad_mesh("zero face area", [](Mesh &m) { m.area[2] = 0.0; });
    bad_mesh("negative cell volume", [](Mesh &m) { m.vol[1] = -1.0; });
    bad_mesh("normal not a unit vector", [](Mesh &m) { m.nrm[0] = 0.9; });
    bad_mesh("non-finite face centroid", [](Mesh &m) { m.fcen[1] = NAN; });
    bad_mesh("non-finite periodic shift", [](Mesh &m) { m.shift[0] = INFINITY; });
    bad_mesh("unknown boundary type", [](Mesh &m) { m.bc[0] = 9; });
    bad_mesh("boundary id without a row", [](Mesh &m) {
        m.fc[1] = -1;
        m.bc[0] = UGKS_BC_WALL;
        m.bcid[0] = 3;
    });
    bad_mesh("cell with too many faces", [](Mesh &m) {
        const double n[2] = {1.0, 0.0}, c[2] = {0.5, 0.5}, s[2] = {0.0, 0.0};
        m.face(0, 1, n, 0.1, c, s, UGKS_BC_INTERIOR, 0);
    });
    bad_mesh("zero cells", [](Mesh &m) { m.nc = 0; });
    {
        std::vector<double> p = p0;
        p[0] = 0.0;
        create_invalid(per, v2, g0, p, "zero initial density");
        p = p0;
        p[3] = -1.0;
        create_invalid(per, v2, g0, p, "negative initial temperature");
    }
    {
        VGrid v = v2;
        v.w[3] = 0.0;
        create_invalid(per, v, g0, p0, "zero velocity weight");
        v = v2;
        v.u[5] = NAN;
        create_invalid(per, v, g0, p0, "non-finite velocity");
        v = v2;
        v.dim = 3;
        create_invalid(per, v, g0, p0, "velocity dimension differs");
    }
    auto bad_gas = [&](const std::string &what, const std::function<void(ugks_gas_t &)> &edit) {
        ugks_gas_t g = g0;
        edit(g);
        create_invalid(per, v2, g, p0, what);
    };
    bad_gas("storage type", [](ugks_gas_t &g) { g.fstore = 7; });
    bad_gas("Prandtl number", [](ugks_gas_t &g) { g.Pr = 0.0; });
    bad_gas("viscosity", [](ugks_gas_t &g) { g.mu_ref = -1.0; });
    bad_gas("CFL number", [](ugks_gas_t &g) { g.cfl = 0.0; });
    bad_gas("limiter constant", [](ugks_gas_t &g) { g.limiter_k = -1.0; });
    bad_gas("memory mode", [](ugks_gas_t &g) { g.mem_mode = 5; });
    bad_gas("chunk", [](ugks_gas_t &g) { g.chunk = -2; });
    bad_gas("sweep", [](ugks_gas_t &g) { g.sweep = 4; });
    bad_gas("negative sweep", [](ugks_gas_t &g) { g.sweep = -1; });
    bad_gas("boundary rows missing", [](ugks_gas_t &g) { g.n_bc = 2; });

    // the static batch refuses before touching the device
    expect(ugks_batch_step_static(nullptr, 1, 1, nullptr) == UGKS_ERR_ARG, "static batch of NULL handles");
    expect(ugks_batch_step_static(nullptr, UGKS_STATIC_BATCH_MAX + 1, 1, nullptr) == UGKS_ERR_ARG,
           "static batch over its limit");

    std::printf("%d checks, %d failed\n", g_checks, g_fail);
    return g_fail ? 1 : 0;
}
