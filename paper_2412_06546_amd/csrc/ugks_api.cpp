// ugks_api.cpp -- host side of the MI355X UGKS library: input validation,
// mesh preprocessing (stencils, least-squares weights, limiter constants),
// device memory, the CFL time step, and the C ABI declared in ugks.h.
#include "../../include/ugks.h"
#include "ugks_internal.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

using namespace ugx;

static_assert(kStaticBatchMax == UGKS_STATIC_BATCH_MAX, "static batch limit of the header and the kernels");

struct ugks {
    int dim = 0, nc = 0, nf = 0, nv = 0, ncomp = 0, fstore = 0, nbc = 0;
    hipStream_t stream = nullptr;
    Params P{};
    void *f[2] = {nullptr, nullptr};
    int cur = 0;
    void *cgeo = nullptr, *fgeo = nullptr, *feq = nullptr;
    double *u = nullptr, *w = nullptr, *bcp = nullptr, *W = nullptr, *q = nullptr, *gW = nullptr, *dW2 = nullptr;
    double *cell_dt = nullptr, *res = nullptr, *u1d = nullptr;
    int *err = nullptr, *kidx = nullptr;
    // surface quantities: stored indices of the wall faces (in the caller's
    // face order), their flux in the last step, and whether a step has run
    // since creation or set_f (f[1 - cur] then holds the f that started it)
    int mem_mode = UGKS_MEM_TWO_BUFFERS;
    void *ring = nullptr;          // in-place mode: one chunk of stage-1 values per cell
    double *mom_part = nullptr;    // moments of the chunks swept so far (in place) or of the stage-1 base (push)
    double *rho_w = nullptr;       // wall densities (in place, push)
    double *mom_s = nullptr;       // push sweep in place: stage-1 moments about U^n summed over the chunks
    // push sweep: colour lists (device cells, host offsets), wall cells,
    // face -> wall ordinal; whether the second buffer holds the stage-1 base
    // of the current f, and whether the last step was a push step (the wall
    // flux of that step is then already in wallF)
    int push = 0, unordered = 0, base_ok = 0, last_push = 0;
    int *colour_cells = nullptr, *wall_cells = nullptr, *wall_index = nullptr;
    int n_wall_cells = 0;
    std::vector<int> colour_off;
    int n_wallf = 0;
    int *wallf = nullptr;
    double *wallF = nullptr, *surf = nullptr;
    int stepped = 0;
    double dt = 0.0;
    long nstep = 0;
    int tensor = 0;
    size_t bytes = 0;
    std::string msg;
    // optional per-launch timing: events around the prologue and the sweep
    int profiling = 0;
    std::vector<hipEvent_t> ev;  // 3 per step: before prologue, before sweep, after sweep
    double prof_ms[2] = {0.0, 0.0};
    long prof_n = 0;
    std::vector<int> perm;     // stored velocity index -> caller's index
    std::vector<int> cell_of;  // stored cell index -> caller's index
    // asynchronous stepping: pinned copies of the error flag and residual,
    // and an event marking the end of the last enqueued steps
    int *h_err = nullptr;
    double *h_res = nullptr;
    hipEvent_t done_ev = nullptr;
    int pending = 0;
};

// text of the last failed create call, per calling thread
static thread_local std::string g_create_error;
// text of the last failed ugks_batch_step_static of the calling thread (a
// fixed buffer: that entry point allocates nothing, not even on failure)
static thread_local char g_static_batch_error[256] = "";

namespace {

struct Fail {
    int code;
    std::string msg;
};

// bfloat16 storage on the host side (same rounding as the device: nearest,
// ties to even, straight from FP64; below the FP32 normal range -> zero)
uint16_t bf16_of(double x)
{
    if (x != x) return 0x7fc0;
    uint64_t u;
    std::memcpy(&u, &x, 8);
    u += 0x00000fffffffffffull + ((u >> 45) & 1ull);
    u &= ~0x00001fffffffffffull;
    double r;
    std::memcpy(&r, &u, 8);
    float f = std::fabs(r) < 1.1754943508222875e-38 ? std::copysign(0.0f, (float)r) : (float)r;
    uint32_t b;
    std::memcpy(&b, &f, 4);
    return (uint16_t)(b >> 16);
}
double double_of_bf16(uint16_t v)
{
    const uint32_t b = (uint32_t)v << 16;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}
size_t fvalue_bytes(int fstore) { return fstore == UGKS_BF16 ? 2 : (fstore == UGKS_F32 ? 4 : 8); }

template <typename T> T *dev_alloc(ugks_t *h, size_t n)
{
    void *p = nullptr;
    size_t b = sizeof(T) * (n ? n : 1);
    if (hipMalloc(&p, b) != hipSuccess) throw Fail{UGKS_ERR_ALLOC, "hipMalloc of " + std::to_string(b) + " bytes failed"};
    h->bytes += b;
    return static_cast<T *>(p);
}

void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) throw Fail{UGKS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e)};
}

void upload(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s), "hipMemcpyAsync H2D");
}

// Separable Gaussians: exp(-lam |u - U|^2) is the product over the axes of
// exp(-lam (u_d - U_d)^2), so it can be tabulated per axis over the distinct
// values that the velocity set's coordinates take on that axis.  That holds
// for Cartesian grids, and equally for octree-refined or ball-restricted
// sets, whose points share few coordinate values per axis.  Returns 1 with
// the axes (the sorted distinct values, x then y [then z]), their counts and
// every velocity's packed axis indices (a | b << 10 | c << 20), when every
// axis has at most 1023 distinct values.
int detect_tensor(int D, int nv, const double *u, int n1d[3], std::vector<double> &axes, std::vector<int> &kidx)
{
    std::vector<double> vals[3];
    for (int d = 0; d < D; ++d) {
        vals[d].resize(nv);
        for (int k = 0; k < nv; ++k) vals[d][k] = u[(size_t)k * D + d];
        std::sort(vals[d].begin(), vals[d].end());
        vals[d].erase(std::unique(vals[d].begin(), vals[d].end()), vals[d].end());
        if (vals[d].size() > 1023) return 0;
    }
    axes.clear();
    for (int d = 0; d < 3; ++d) {
        n1d[d] = d < D ? (int)vals[d].size() : 0;
        if (d < D) axes.insert(axes.end(), vals[d].begin(), vals[d].end());
    }
    kidx.assign(nv, 0);
    for (int k = 0; k < nv; ++k)
        for (int d = 0; d < D; ++d) {
            const double x = u[(size_t)k * D + d];
            const int a = (int)(std::lower_bound(vals[d].begin(), vals[d].end(), x) - vals[d].begin());
            kidx[k] |= a << (10 * d);
        }
    return 1;
}

// Velocities are stored ordered by direction, so the 64 lanes of a wavefront
// hold nearly parallel velocities and agree on the upwind side of almost
// every face (only wavefronts straddling a face's tangent line diverge).
// 2D: by polar angle, then speed.  3D: by polar band, then azimuth
// (alternating direction band to band), then speed.
std::vector<int> direction_order(int D, int nv, const double *u)
{
    std::vector<int> idx(nv);
    std::vector<double> k1(nv), k2(nv), k3(nv);
    const int nb = D == 3 ? std::max(1, (int)std::lround(std::sqrt(nv / 64.0))) : 1;
    for (int k = 0; k < nv; ++k) {
        idx[k] = k;
        const double *v = u + (size_t)k * D;
        double s2 = 0.0;
        for (int d = 0; d < D; ++d) s2 += v[d] * v[d];
        const double az = std::atan2(v[1], v[0]);
        if (D == 2) {
            k1[k] = 0.0;
            k2[k] = az;
        } else {
            const double r = std::sqrt(s2);
            const int band = r > 0.0 ? std::min(nb - 1, (int)(std::acos(std::max(-1.0, std::min(1.0, v[2] / r))) / M_PI * nb)) : 0;
            k1[k] = band;
            k2[k] = (band & 1) ? -az : az;
        }
        k3[k] = s2;
    }
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        if (k1[a] != k1[b]) return k1[a] < k1[b];
        if (k2[a] != k2[b]) return k2[a] < k2[b];
        return k3[a] < k3[b];
    });
    return idx;
}

// Caller's face records checked before anything is indexed by them.
void validate_faces(const ugks_mesh_t *m, int nbc)
{
    const int nc = m->n_cells;
    for (int f = 0; f < m->n_faces; ++f) {
        const int l = m->face_cells[2 * f], r = m->face_cells[2 * f + 1];
        const int bc = m->face_bc ? m->face_bc[f] : UGKS_BC_INTERIOR;
        const int bid = m->face_bc_id ? m->face_bc_id[f] : 0;
        if (l < 0 || l >= nc || r >= nc || r < -1) throw Fail{UGKS_ERR_ARG, "face " + std::to_string(f) + ": cell index out of range"};
        if ((r < 0) != (bc != UGKS_BC_INTERIOR))
            throw Fail{UGKS_ERR_ARG, "face " + std::to_string(f) + ": boundary type does not match its cells"};
        if (bc < 0 || bc > 3) throw Fail{UGKS_ERR_ARG, "face " + std::to_string(f) + ": unknown boundary type"};
        if (bc != UGKS_BC_INTERIOR && bc != UGKS_BC_OUTFLOW && (bid < 0 || bid >= nbc))
            throw Fail{UGKS_ERR_ARG, "face " + std::to_string(f) + ": boundary state index out of range"};
        if (!(m->face_area[f] > 0.0)) throw Fail{UGKS_ERR_ARG, "face " + std::to_string(f) + ": non-positive area"};
        double n2 = 0.0;
        bool finite = true;
        for (int d = 0; d < m->dim; ++d) {
            const double nd = m->face_normal[(size_t)f * m->dim + d];
            n2 += nd * nd;
            finite = finite && std::isfinite(m->face_centroid[(size_t)f * m->dim + d]) &&
                     (!m->face_shift || std::isfinite(m->face_shift[(size_t)f * m->dim + d]));
        }
        if (!(std::fabs(n2 - 1.0) < 1e-6)) throw Fail{UGKS_ERR_ARG, "face " + std::to_string(f) + ": normal is not a unit vector"};
        if (!finite) throw Fail{UGKS_ERR_ARG, "face " + std::to_string(f) + ": non-finite centroid or periodic shift"};
    }
    for (int c = 0; c < nc; ++c)
        for (int d = 0; d < m->dim; ++d)
            if (!std::isfinite(m->cell_centroid[(size_t)c * m->dim + d]))
                throw Fail{UGKS_ERR_ARG, "cell " + std::to_string(c) + ": non-finite centroid"};
}

// The library stores cells along a Morton (Z-order) curve through their
// centroids, so that a run of consecutive stored cells -- the workgroups
// that one XCD, and so one L2, receives -- is a compact patch of the mesh
// whatever the caller's numbering; neighbours' f slabs are then re-read from
// L2 rather than HBM.  Faces are stored sorted by their first stored cell,
// which keeps the face prologue's cell reads local as well.  The relabelled
// mesh owns its arrays; cell_of/face_of map stored indices to the caller's.
struct StoredMesh {
    std::vector<int> cell_of, face_of, pos_of;
    std::vector<double> vol, cen, nrm, area, fcen, shift;
    std::vector<int> fcells, bc, bcid;
    ugks_mesh_t mesh{};
};

void relabel(const ugks_mesh_t *m, StoredMesh &S)
{
    const int D = m->dim, nc = m->n_cells, nf = m->n_faces;
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    for (int c = 0; c < nc; ++c)
        for (int d = 0; d < D; ++d) {
            lo[d] = std::min(lo[d], m->cell_centroid[(size_t)c * D + d]);
            hi[d] = std::max(hi[d], m->cell_centroid[(size_t)c * D + d]);
        }
    const int bits = 21;
    const double top = (double)((1u << bits) - 1);
    std::vector<std::pair<unsigned long long, int>> key(nc);
    for (int c = 0; c < nc; ++c) {
        unsigned long long code = 0;
        for (int d = 0; d < D; ++d) {
            const double span = hi[d] - lo[d];
            const double x = span > 0.0 ? (m->cell_centroid[(size_t)c * D + d] - lo[d]) / span : 0.0;
            const unsigned long long qd = (unsigned long long)std::min(top, std::max(0.0, std::floor(x * top)));
            for (int b = 0; b < bits; ++b) code |= ((qd >> b) & 1ull) << (b * D + d);
        }
        key[c] = {code, c};
    }
    std::sort(key.begin(), key.end());
    S.cell_of.resize(nc);
    S.pos_of.resize(nc);
    for (int i = 0; i < nc; ++i) {
        S.cell_of[i] = key[i].second;
        S.pos_of[key[i].second] = i;
    }
    std::vector<std::pair<long long, int>> fkey(nf);
    for (int f = 0; f < nf; ++f) {
        const int l = S.pos_of[m->face_cells[2 * f]], r = m->face_cells[2 * f + 1];
        const int first = r >= 0 ? std::min(l, S.pos_of[r]) : l;
        fkey[f] = {(long long)first, f};
    }
    std::sort(fkey.begin(), fkey.end());
    S.face_of.resize(nf);
    for (int i = 0; i < nf; ++i) S.face_of[i] = fkey[i].second;

    S.vol.resize(nc);
    S.cen.resize((size_t)nc * D);
    for (int i = 0; i < nc; ++i) {
        const int c = S.cell_of[i];
        S.vol[i] = m->cell_volume[c];
        for (int d = 0; d < D; ++d) S.cen[(size_t)i * D + d] = m->cell_centroid[(size_t)c * D + d];
    }
    S.nrm.resize((size_t)nf * D);
    S.fcen.resize((size_t)nf * D);
    S.shift.assign((size_t)nf * D, 0.0);
    S.area.resize(nf);
    S.fcells.resize(2 * (size_t)nf);
    S.bc.resize(nf);
    S.bcid.resize(nf);
    for (int i = 0; i < nf; ++i) {
        const int f = S.face_of[i], r = m->face_cells[2 * f + 1];
        S.fcells[2 * i] = S.pos_of[m->face_cells[2 * f]];
        S.fcells[2 * i + 1] = r >= 0 ? S.pos_of[r] : -1;
        S.area[i] = m->face_area[f];
        S.bc[i] = m->face_bc ? m->face_bc[f] : UGKS_BC_INTERIOR;
        S.bcid[i] = m->face_bc_id ? m->face_bc_id[f] : 0;
        for (int d = 0; d < D; ++d) {
            S.nrm[(size_t)i * D + d] = m->face_normal[(size_t)f * D + d];
            S.fcen[(size_t)i * D + d] = m->face_centroid[(size_t)f * D + d];
            if (m->face_shift) S.shift[(size_t)i * D + d] = m->face_shift[(size_t)f * D + d];
        }
    }
    S.mesh = *m;
    S.mesh.cell_volume = S.vol.data();
    S.mesh.cell_centroid = S.cen.data();
    S.mesh.face_cells = S.fcells.data();
    S.mesh.face_normal = S.nrm.data();
    S.mesh.face_area = S.area.data();
    S.mesh.face_centroid = S.fcen.data();
    S.mesh.face_shift = S.shift.data();
    S.mesh.face_bc = S.bc.data();
    S.mesh.face_bc_id = S.bcid.data();
}

template <int D>
void build_geometry(const StoredMesh &S, std::vector<CellGeo<D>> &cg, std::vector<FaceGeo<D>> &fgv, double limiter_k)
{
    const ugks_mesh_t *m = &S.mesh;
    auto cname = [&](int c) { return "cell " + std::to_string(S.cell_of[c]); };
    auto fname = [&](int f) { return "face " + std::to_string(S.face_of[f]); };
    constexpr int MF = Dim<D>::MF;
    const int nc = m->n_cells, nf = m->n_faces;
    cg.assign(nc, CellGeo<D>{});
    fgv.assign(nf, FaceGeo<D>{});
    std::vector<int> slot_count(nc, 0);
    for (int f = 0; f < nf; ++f) {
        const int l = m->face_cells[2 * f], r = m->face_cells[2 * f + 1];
        const int bc = m->face_bc[f], bid = m->face_bc_id[f];
        FaceGeo<D> &F = fgv[f];
        F.l = l;
        F.r = r;
        F.bc = bc;
        F.bcid = bid;
        F.area = m->face_area[f];
        for (int d = 0; d < D; ++d) {
            const double sh = m->face_shift[(size_t)f * D + d];
            F.n[d] = m->face_normal[(size_t)f * D + d];
            F.dl[d] = m->face_centroid[(size_t)f * D + d] - m->cell_centroid[(size_t)l * D + d];
            F.dr[d] = r >= 0 ? m->face_centroid[(size_t)f * D + d] - sh - m->cell_centroid[(size_t)r * D + d] : 0.0;
        }
        for (int s = 0; s < 2; ++s) {
            const int c = s == 0 ? l : r;
            if (c < 0) continue;
            const int j = slot_count[c]++;
            if (j >= MF) throw Fail{UGKS_ERR_ARG, cname(c) + " has more than " + std::to_string(MF) + " faces"};
            CellGeo<D> &g = cg[c];
            g.face[j] = f;
            g.side[j] = s;
            g.nb[j] = s == 0 ? r : l;
            for (int d = 0; d < D; ++d) g.dvec[j][d] = s == 0 ? F.dl[d] : F.dr[d];
        }
    }
    for (int c = 0; c < nc; ++c) {
        CellGeo<D> &g = cg[c];
        g.nf = slot_count[c];
        if (g.nf < D + 1) throw Fail{UGKS_ERR_ARG, cname(c) + " has fewer than dim+1 faces"};
        if (!(m->cell_volume[c] > 0.0)) throw Fail{UGKS_ERR_ARG, cname(c) + ": non-positive volume"};
        g.inv_vol = 1.0 / m->cell_volume[c];
        const double kh = limiter_k * std::pow(m->cell_volume[c], 1.0 / D);
        g.eps2 = kh * kh * kh;
        for (int j = g.nf; j < MF; ++j) {
            g.face[j] = 0;
            g.nb[j] = -1;
            g.back[j] = 0;
            g.side[j] = 0;
        }
        // least-squares normal matrix over face neighbours (periodic images)
        double G[9] = {0}, dn[MF][D];
        for (int j = 0; j < g.nf; ++j) {
            const int n = g.nb[j];
            for (int d = 0; d < D; ++d) dn[j][d] = 0.0;
            if (n < 0) continue;
            const int f = g.face[j];
            for (int d = 0; d < D; ++d) {
                const double sh = m->face_shift[(size_t)f * D + d];
                dn[j][d] = m->cell_centroid[(size_t)n * D + d] + (g.side[j] == 0 ? sh : -sh) - m->cell_centroid[(size_t)c * D + d];
            }
            for (int a = 0; a < D; ++a)
                for (int b = 0; b < D; ++b) G[a * D + b] += dn[j][a] * dn[j][b];
            // slot of the same face in the neighbour (the opposite side)
            const CellGeo<D> &gn = cg[n];
            int bj = -1;
            for (int t = 0; t < slot_count[n]; ++t)
                if (gn.face[t] == f && gn.side[t] != g.side[j]) bj = t;
            if (bj < 0) throw Fail{UGKS_ERR_ARG, "inconsistent face adjacency at " + fname(f)};
            g.back[j] = bj;
        }
        // A stencil with no more neighbours than dimensions (a triangle or a
        // tetrahedron with a boundary face) is an interpolation, not a
        // least-squares fit: its extrapolation to the other faces leans
        // downwind and the second-order transport is unstable there, so
        // such a cell keeps a zero gradient, as a degenerate one does.
        int n_nb = 0;
        for (int j = 0; j < g.nf; ++j) n_nb += g.nb[j] >= 0;
        double Gi[9] = {0}, tr = 0.0, det;
        for (int a = 0; a < D; ++a) tr += G[a * D + a];
        const double tol = n_nb > D ? 1e-10 * std::pow(tr / D, D) : HUGE_VAL;
        if (D == 2) {
            det = G[0] * G[3] - G[1] * G[2];
            if (det > tol) {
                Gi[0] = G[3] / det;
                Gi[1] = -G[1] / det;
                Gi[2] = -G[2] / det;
                Gi[3] = G[0] / det;
            }
        } else {
            const double c00 = G[4] * G[8] - G[5] * G[7], c01 = G[5] * G[6] - G[3] * G[8], c02 = G[3] * G[7] - G[4] * G[6];
            det = G[0] * c00 + G[1] * c01 + G[2] * c02;
            if (det > tol) {
                Gi[0] = c00 / det;
                Gi[1] = (G[2] * G[7] - G[1] * G[8]) / det;
                Gi[2] = (G[1] * G[5] - G[2] * G[4]) / det;
                Gi[3] = c01 / det;
                Gi[4] = (G[0] * G[8] - G[2] * G[6]) / det;
                Gi[5] = (G[2] * G[3] - G[0] * G[5]) / det;
                Gi[6] = c02 / det;
                Gi[7] = (G[1] * G[6] - G[0] * G[7]) / det;
                Gi[8] = (G[0] * G[4] - G[1] * G[3]) / det;
            }
        }
        for (int j = 0; j < MF; ++j)
            for (int a = 0; a < D; ++a) {
                double s = 0.0;
                if (j < g.nf)
                    for (int b = 0; b < D; ++b) s += Gi[a * D + b] * dn[j][b];
                g.lsq[j][a] = s;
            }
        for (int j = 0; j < MF; ++j)
            g.nb_inv_vol[j] = (j < g.nf && g.nb[j] >= 0) ? 1.0 / m->cell_volume[g.nb[j]] : 0.0;
    }
}

// Colours of the push sweep: no two cells of a colour are neighbours or
// share a neighbour (greedy distance-2 colouring in stored order); the
// cells grouped by colour, stored order within a colour, and the offsets.
template <int D>
void push_colours(const std::vector<CellGeo<D>> &cg, std::vector<int> &cells, std::vector<int> &off)
{
    const int nc = (int)cg.size();
    std::vector<int> colour(nc, -1), stamp;
    int ncol = 0;
    for (int c = 0; c < nc; ++c) {
        auto mark = [&](int d) {
            if (d >= 0 && colour[d] >= 0) stamp[colour[d]] = c;
        };
        for (int j = 0; j < cg[c].nf; ++j) {
            const int n = cg[c].nb[j];
            if (n < 0) continue;
            mark(n);
            for (int t = 0; t < cg[n].nf; ++t) mark(cg[n].nb[t]);
        }
        int k = 0;
        while (k < ncol && stamp[k] == c) ++k;
        if (k == ncol) {
            ++ncol;
            stamp.push_back(-1);
        }
        colour[c] = k;
    }
    off.assign(ncol + 1, 0);
    for (int c = 0; c < nc; ++c) ++off[colour[c] + 1];
    for (int k = 0; k < ncol; ++k) off[k + 1] += off[k];
    cells.assign(nc, 0);
    std::vector<int> at(off.begin(), off.end() - 1);
    for (int c = 0; c < nc; ++c) cells[at[colour[c]]++] = c;
}

template <int D> void create_d(ugks_t *h, const StoredMesh &S, const ugks_gas_t *gas)
{
    std::vector<CellGeo<D>> cg;
    std::vector<FaceGeo<D>> fgv;
    build_geometry<D>(S, cg, fgv, gas->limiter_k);
    if (h->push) {
        std::vector<int> cells;
        if (h->unordered) {  // one class: every cell, in stored order
            cells.resize(cg.size());
            for (size_t c = 0; c < cells.size(); ++c) cells[c] = (int)c;
            h->colour_off = {0, (int)cg.size()};
        } else {
            push_colours<D>(cg, cells, h->colour_off);
        }
        h->colour_cells = dev_alloc<int>(h, cells.size());
        upload(h->colour_cells, cells.data(), sizeof(int) * cells.size(), h->stream);
        std::vector<int> wc;
        for (int c = 0; c < (int)cg.size(); ++c) {
            bool w = false;
            for (int j = 0; j < cg[c].nf; ++j) w = w || fgv[cg[c].face[j]].bc == UGKS_BC_WALL;
            if (w) wc.push_back(c);
        }
        size_t nwallf = 0;
        for (const auto &F : fgv) nwallf += F.bc == UGKS_BC_WALL;
        h->n_wall_cells = (int)wc.size();
        h->wall_cells = dev_alloc<int>(h, nwallf);  // at most one cell per wall face
        if (!wc.empty()) upload(h->wall_cells, wc.data(), sizeof(int) * wc.size(), h->stream);
    }
    h->cgeo = dev_alloc<CellGeo<D>>(h, cg.size());
    h->fgeo = dev_alloc<FaceGeo<D>>(h, fgv.size());
    h->feq = dev_alloc<FaceEq<D>>(h, fgv.size());
    upload(h->cgeo, cg.data(), sizeof(CellGeo<D>) * cg.size(), h->stream);
    upload(h->fgeo, fgv.data(), sizeof(FaceGeo<D>) * fgv.size(), h->stream);
    hip_check(hipMemsetAsync(h->feq, 0, sizeof(FaceEq<D>) * fgv.size(), h->stream), "hipMemsetAsync");
    hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
}

// Device bytes a handle owns once created (the same sizes ugks_create
// allocates; the temporary initial-state buffer is not counted).
template <typename T> size_t nbytes(size_t n) { return sizeof(T) * (n ? n : 1); }
// in-place mode: velocities per chunk (0 asks for the default) and chunk count
int chunk_of(int chunk, int nv) { return std::min(chunk > 0 ? chunk : UGKS_DEFAULT_CHUNK, nv); }
int nchunk_of(int chunk, int nv) { return (nv + chunk - 1) / chunk; }

// whether a handle sweeps by pushing each face flux once (else gathering).
// Automatic choice: push, except for 2D with FP64 f in two buffers, where
// gathering is faster on MI355X (2D hypersonic cylinder, 20,000 cells x
// 3,600 velocities: 3.2 against 4.2 ms per step; FP32 f 2.7 push against 2.9
// gather; the 3D lifting body 178 push against 295 ms gather in FP64).
// BF16 f pushes only when asked: its accumulator (the second buffer, or the
// ring in place) holds FP32 stage-1 sums, 2 more bytes per value.
bool asks_push(const ugks_gas_t *gas) { return gas->sweep == UGKS_SWEEP_PUSH || gas->sweep == UGKS_SWEEP_PUSH_UNORDERED; }
bool uses_push(int dim, const ugks_gas_t *gas)
{
    if (gas->sweep == UGKS_SWEEP_GATHER) return false;
    if (gas->fstore == UGKS_BF16) return asks_push(gas);
    if (asks_push(gas) || gas->mem_mode == UGKS_MEM_IN_PLACE) return true;
    return !(dim == 2 && gas->fstore == UGKS_F64);
}
// the push sweep's running moment sums about U^n, per cell (in place)
int shift_moments(int D) { return D == 2 ? 11 : 13; }

size_t plan_bytes(int D, size_t nc, size_t nf, size_t nv, int nbc, int fstore, size_t ntab, size_t nwallf,
                  int mem_mode = UGKS_MEM_TWO_BUFFERS, int chunk = 0, bool push = false)
{
    const size_t NW = D + 2, ncomp = D == 2 ? 2 : 1;
    size_t b = D == 2 ? nbytes<CellGeo<2>>(nc) + nbytes<FaceGeo<2>>(nf) + nbytes<FaceEq<2>>(nf)
                      : nbytes<CellGeo<3>>(nc) + nbytes<FaceGeo<3>>(nf) + nbytes<FaceEq<3>>(nf);
    b += nbytes<double>(D * nv) + nbytes<double>(nv) + nbytes<double>((size_t)std::max(1, nbc) * NW);
    b += nbytes<double>(nc * NW) + nbytes<double>(nc * D) + nbytes<double>(nc * NW * D) + nbytes<double>(nc * NW);
    b += nbytes<double>(nc) + nbytes<double>(NW * (1 + (size_t)residual_groups((int)nc))) + nbytes<int>(2);
    if (ntab) b += nbytes<double>(ntab) + nbytes<int>(nv);
    if (mem_mode == UGKS_MEM_IN_PLACE) {
        const int ch = chunk_of(chunk, (int)nv);
        b += nc * ncomp * nv * fvalue_bytes(fstore);                      // f
        b += nbytes<char>(nc * ncomp * (size_t)ch * (push && fstore == UGKS_BF16 ? 4 : fvalue_bytes(fstore)));  // ring
        b += nbytes<double>(nc * (size_t)NW) + nbytes<double>(nc * (D == 2 ? Dim<2>::MF : Dim<3>::MF));
    } else {  // f, and the second buffer (FP32 stage-1 sums when BF16 f pushes)
        b += nc * ncomp * nv * (fvalue_bytes(fstore) + (push && fstore == UGKS_BF16 ? 4 : fvalue_bytes(fstore)));
    }
    if (push) {  // colour lists, wall cells, face -> wall ordinal
        b += nbytes<int>(nc) + nbytes<int>(nwallf) + nbytes<int>(nf);
        if (mem_mode == UGKS_MEM_IN_PLACE)  // the running moments about U^n
            b += nbytes<double>(nc * (size_t)shift_moments(D));
        else  // base moments, wall densities
            b += nbytes<double>(nc * NW) + nbytes<double>(nc * (D == 2 ? Dim<2>::MF : Dim<3>::MF));
    }
    b += nbytes<int>(nwallf) + nbytes<double>(nwallf * NW) + nbytes<double>(nwallf * 6);
    return b;
}

int fail(ugks_t *h, const Fail &e)
{
    if (h) h->msg = e.msg;
    else {
        g_create_error = e.msg;
        g_static_batch_error[0] = 0;
    }
    return e.code;
}

// err[1] holds the lowest stored index of a failing cell; the message names
// the caller's index.
std::string nonphysical_message(const ugks_t *h, int stored)
{
    const int c = stored >= 0 && stored < h->nc ? h->cell_of[stored] : stored;
    return "non-physical state (rho <= 0, T <= 0 or non-finite) at cell " + std::to_string(c);
}

// pinned copies of the flag and residual, and the completion event, for
// asynchronous stepping (allocated on first use)
void ensure_async(ugks_t *h)
{
    if (h->h_err) return;
    hip_check(hipHostMalloc((void **)&h->h_err, 2 * sizeof(int), hipHostMallocDefault), "hipHostMalloc");
    hip_check(hipHostMalloc((void **)&h->h_res, (h->dim + 2) * sizeof(double), hipHostMallocDefault), "hipHostMalloc");
    hip_check(hipEventCreateWithFlags(&h->done_ev, hipEventDisableTiming), "hipEventCreate");
}

// after the steps and the residual kernel: copy flag and residual to pinned
// memory, mark the end, and leave the handle pending until ugks_poll
void finish_async(ugks_t *h)
{
    hip_check(hipMemcpyAsync(h->h_err, h->err, 2 * sizeof(int), hipMemcpyDeviceToHost, h->stream), "copy flag");
    hip_check(hipMemcpyAsync(h->h_res, h->res, (h->dim + 2) * sizeof(double), hipMemcpyDeviceToHost, h->stream),
              "copy residual");
    hip_check(hipEventRecord(h->done_ev, h->stream), "hipEventRecord");
    h->pending = 1;
}

void release(ugks_t *h)
{
    if (h->h_err) (void)hipHostFree(h->h_err);
    if (h->h_res) (void)hipHostFree(h->h_res);
    if (h->done_ev) (void)hipEventDestroy(h->done_ev);
    void *ptrs[] = {h->f[0], h->f[1], h->cgeo, h->fgeo, h->feq, h->u, h->w, h->bcp, h->W, h->q, h->gW, h->dW2,
                    h->cell_dt, h->res, h->err, h->u1d, h->kidx, h->wallf, h->wallF, h->surf, h->ring, h->mom_part, h->rho_w,
                    h->mom_s, h->colour_cells, h->wall_cells, h->wall_index};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
}

}  // namespace

extern "C" int ugks_create(const ugks_mesh_t *mesh, const ugks_vgrid_t *vgrid, const ugks_gas_t *gas,
                           const double *prim0, void *stream, ugks_t **out)
{
    if (!out) {
        g_create_error = "out is NULL";
        return UGKS_ERR_ARG;
    }
    *out = nullptr;
    ugks_t *h = new (std::nothrow) ugks_t();
    if (!h) {
        g_create_error = "host allocation failed";
        return UGKS_ERR_ALLOC;
    }
    double *prim_d = nullptr;  // initial state on the device, freed before returning
    try {
        if (!mesh || !vgrid || !gas || !prim0) throw Fail{UGKS_ERR_ARG, "NULL argument"};
        const int D = mesh->dim;
        if (D != 2 && D != 3) throw Fail{UGKS_ERR_ARG, "dim must be 2 or 3"};
        if (vgrid->dim != D) throw Fail{UGKS_ERR_ARG, "velocity grid and mesh dimensions differ"};
        if (mesh->n_cells <= 0 || mesh->n_faces <= 0 || vgrid->n_vel <= 0)
            throw Fail{UGKS_ERR_ARG, "empty mesh or velocity grid"};
        if (vgrid->n_vel > 16384) throw Fail{UGKS_ERR_ARG, "more than 16384 discrete velocities"};
        // per-cell launches of 256 threads must stay below 2^32 work-items
        if (mesh->n_cells > 16000000) throw Fail{UGKS_ERR_ARG, "more than 16,000,000 cells"};
        if (!mesh->cell_volume || !mesh->cell_centroid || !mesh->face_cells || !mesh->face_normal || !mesh->face_area ||
            !mesh->face_centroid || !vgrid->u || !vgrid->w)
            throw Fail{UGKS_ERR_ARG, "NULL mesh or velocity array"};
        if (gas->fstore != UGKS_F64 && gas->fstore != UGKS_F32 && gas->fstore != UGKS_BF16)
            throw Fail{UGKS_ERR_ARG, "fstore must be UGKS_F64, UGKS_F32 or UGKS_BF16"};
        if (!(gas->Pr > 0.0) || !(gas->mu_ref > 0.0) || !(gas->cfl > 0.0) || gas->limiter_k < 0.0)
            throw Fail{UGKS_ERR_ARG, "Pr, mu_ref and cfl must be positive, limiter_k non-negative"};
        if (gas->n_bc < 0 || (gas->n_bc > 0 && !gas->bc_prim)) throw Fail{UGKS_ERR_ARG, "bc_prim missing"};
        if (gas->mem_mode != UGKS_MEM_TWO_BUFFERS && gas->mem_mode != UGKS_MEM_IN_PLACE)
            throw Fail{UGKS_ERR_ARG, "mem_mode must be UGKS_MEM_TWO_BUFFERS or UGKS_MEM_IN_PLACE"};
        if (gas->chunk < 0) throw Fail{UGKS_ERR_ARG, "chunk must be >= 0"};
        if (gas->sweep < UGKS_SWEEP_AUTO || gas->sweep > UGKS_SWEEP_PUSH_UNORDERED)
            throw Fail{UGKS_ERR_ARG,
                       "sweep must be UGKS_SWEEP_AUTO, UGKS_SWEEP_GATHER, UGKS_SWEEP_PUSH or UGKS_SWEEP_PUSH_UNORDERED"};
        h->push = uses_push(D, gas) ? 1 : 0;
        h->unordered = gas->sweep == UGKS_SWEEP_PUSH_UNORDERED ? 1 : 0;
        for (int k = 0; k < vgrid->n_vel; ++k) {
            bool ok = vgrid->w[k] > 0.0 && std::isfinite(vgrid->w[k]);
            for (int d = 0; d < D; ++d) ok = ok && std::isfinite(vgrid->u[(size_t)k * D + d]);
            if (!ok) throw Fail{UGKS_ERR_ARG, "velocity " + std::to_string(k) + ": non-finite point or non-positive weight"};
        }
        h->dim = D;
        h->nc = mesh->n_cells;
        h->nf = mesh->n_faces;
        h->nv = vgrid->n_vel;
        h->ncomp = D == 2 ? 2 : 1;
        h->fstore = gas->fstore;
        h->nbc = gas->n_bc;
        h->stream = static_cast<hipStream_t>(stream);
        for (int i = 0; i < h->nc; ++i) {
            const double *p = prim0 + (size_t)i * (D + 2);
            if (!(p[0] > 0.0) || !(p[D + 1] > 0.0)) throw Fail{UGKS_ERR_ARG, "prim0: rho and T must be positive"};
        }
        validate_faces(mesh, h->nbc);
        StoredMesh S;
        relabel(mesh, S);
        h->cell_of = S.cell_of;
        if (D == 2) create_d<2>(h, S, gas);
        else create_d<3>(h, S, gas);
        int n1d[3] = {0, 0, 0};
        std::vector<double> axes;
        std::vector<int> kidx;
        h->tensor = detect_tensor(D, h->nv, vgrid->u, n1d, axes, kidx);
        // the per-workgroup Gaussian tables must fit in LDS next to the rest
        if (h->tensor && (size_t)(Dim<3>::MF + 1) * axes.size() * sizeof(double) > 48 * 1024) h->tensor = 0;

        const size_t nv = h->nv, nc = h->nc;
        h->perm = direction_order(D, h->nv, vgrid->u);
        std::vector<double> uT((size_t)D * nv), wP(nv);
        for (size_t k = 0; k < nv; ++k) {
            const size_t ku = h->perm[k];
            for (int d = 0; d < D; ++d) uT[(size_t)d * nv + k] = vgrid->u[ku * D + d];
            wP[k] = vgrid->w[ku];
        }
        if (h->tensor) {
            std::vector<int> kp(nv);
            for (size_t k = 0; k < nv; ++k) kp[k] = kidx[h->perm[k]];
            kidx.swap(kp);
        }
        h->u = dev_alloc<double>(h, uT.size());
        h->w = dev_alloc<double>(h, nv);
        h->bcp = dev_alloc<double>(h, (size_t)std::max(1, h->nbc) * (D + 2));
        h->W = dev_alloc<double>(h, nc * (D + 2));
        h->q = dev_alloc<double>(h, nc * D);
        h->gW = dev_alloc<double>(h, nc * (D + 2) * D);
        h->dW2 = dev_alloc<double>(h, nc * (D + 2));
        h->cell_dt = dev_alloc<double>(h, nc);
        h->res = dev_alloc<double>(h, (D + 2) * (1 + (size_t)residual_groups((int)nc)));
        h->err = dev_alloc<int>(h, 2);
        {
            std::vector<std::pair<int, int>> wf;  // (caller's face, stored face)
            for (int f = 0; f < h->nf; ++f)
                if (S.bc[f] == UGKS_BC_WALL) wf.push_back({S.face_of[f], f});
            std::sort(wf.begin(), wf.end());
            std::vector<int> list;
            for (auto &x : wf) list.push_back(x.second);
            h->n_wallf = (int)list.size();
            h->wallf = dev_alloc<int>(h, list.size());
            h->wallF = dev_alloc<double>(h, list.size() * (D + 2));
            h->surf = dev_alloc<double>(h, list.size() * 6);
            if (!list.empty()) upload(h->wallf, list.data(), sizeof(int) * list.size(), h->stream);
            if (h->push) {
                std::vector<int> widx(h->nf, -1);
                for (size_t t = 0; t < list.size(); ++t) widx[list[t]] = (int)t;
                h->wall_index = dev_alloc<int>(h, widx.size());
                upload(h->wall_index, widx.data(), sizeof(int) * widx.size(), h->stream);
            }
            if (h->push && gas->mem_mode == UGKS_MEM_TWO_BUFFERS) {
                h->mom_part = dev_alloc<double>(h, nc * (size_t)(D + 2));
                h->rho_w = dev_alloc<double>(h, nc * (size_t)(D == 2 ? Dim<2>::MF : Dim<3>::MF));
                hip_check(hipMemsetAsync(h->rho_w, 0, sizeof(double) * nc * (D == 2 ? Dim<2>::MF : Dim<3>::MF),
                                         h->stream), "hipMemsetAsync");
            }
        }
        if (h->tensor) {
            h->u1d = dev_alloc<double>(h, axes.size());
            h->kidx = dev_alloc<int>(h, kidx.size());
            upload(h->u1d, axes.data(), sizeof(double) * axes.size(), h->stream);
            upload(h->kidx, kidx.data(), sizeof(int) * kidx.size(), h->stream);
        }
        prim_d = dev_alloc<double>(h, nc * (D + 2));
        const size_t fbytes = nc * h->ncomp * nv * fvalue_bytes(h->fstore);
        h->mem_mode = gas->mem_mode;
        for (int b = 0; b < (h->mem_mode == UGKS_MEM_IN_PLACE ? 1 : 2); ++b) {
            // the push sweep of BF16 f keeps FP32 stage-1 sums in the second
            // buffer (f stays in the first: push steps never swap them)
            const size_t nb = b == 1 && h->push && h->fstore == UGKS_BF16 ? nc * h->ncomp * nv * sizeof(float) : fbytes;
            if (hipMalloc(&h->f[b], nb) != hipSuccess)
                throw Fail{UGKS_ERR_ALLOC, "hipMalloc of f (" + std::to_string(nb) + " bytes) failed"};
            h->bytes += nb;
        }
        int chunk = 0, nchunk = 0;
        if (h->mem_mode == UGKS_MEM_IN_PLACE) {
            chunk = chunk_of(gas->chunk, h->nv);
            nchunk = nchunk_of(chunk, h->nv);
            // FP32 stage-1 sums when BF16 f takes the push sweep
            h->ring = dev_alloc<char>(h, nc * h->ncomp * (size_t)chunk *
                                             (h->push && h->fstore == UGKS_BF16 ? sizeof(float) : fvalue_bytes(h->fstore)));
            h->mom_part = dev_alloc<double>(h, nc * (size_t)(D + 2));
            h->rho_w = dev_alloc<double>(h, nc * (size_t)(D == 2 ? Dim<2>::MF : Dim<3>::MF));
            hip_check(hipMemsetAsync(h->rho_w, 0, sizeof(double) * nc * (D == 2 ? Dim<2>::MF : Dim<3>::MF),
                                     h->stream), "hipMemsetAsync");
            if (h->push) h->mom_s = dev_alloc<double>(h, nc * (size_t)shift_moments(D));
        }
        upload(h->u, uT.data(), sizeof(double) * uT.size(), h->stream);
        upload(h->w, wP.data(), sizeof(double) * nv, h->stream);
        if (h->nbc) upload(h->bcp, gas->bc_prim, sizeof(double) * h->nbc * (D + 2), h->stream);
        std::vector<double> primS(nc * (D + 2));
        for (size_t i = 0; i < nc; ++i)
            for (int m = 0; m < D + 2; ++m) primS[i * (D + 2) + m] = prim0[(size_t)h->cell_of[i] * (D + 2) + m];
        upload(prim_d, primS.data(), sizeof(double) * nc * (D + 2), h->stream);
        const int err0[2] = {0, 0x7fffffff};
        upload(h->err, err0, sizeof(err0), h->stream);

        Params &P = h->P;
        P.dim = D;
        P.fstore = h->fstore;
        P.nc = h->nc;
        P.nf = h->nf;
        P.nv = h->nv;
        P.Pr = gas->Pr;
        P.omega = gas->omega;
        P.mu_ref = gas->mu_ref;
        P.limiter = gas->limiter ? 1 : 0;
        P.cgeo = h->cgeo;
        P.fgeo = h->fgeo;
        P.feq = h->feq;
        P.u = h->u;
        P.w = h->w;
        P.bc_prim = h->bcp;
        P.W = h->W;
        P.q = h->q;
        P.gW = h->gW;
        P.dW2 = h->dW2;
        P.err = h->err;
        P.u1d = h->u1d;
        P.kidx = h->kidx;
        for (int d = 0; d < 3; ++d) P.n1d[d] = h->tensor ? n1d[d] : 0;
        P.ntab = h->tensor ? (int)axes.size() : 0;
        P.ring = h->ring;
        P.chunk = chunk;
        P.nchunk = nchunk;
        P.mom_part = h->mom_part;
        P.rho_w = h->rho_w;
        P.wall_index = h->wall_index;
        P.wflux = h->wallF;
        P.mom_s = h->mom_s;

        // time step (Algorithm 1's first step), fixed for the run
        hip_check(launch_cfl(P, h->cell_dt, h->stream), "k_cfl launch");
        std::vector<double> cdt(nc);
        hip_check(hipMemcpyAsync(cdt.data(), h->cell_dt, sizeof(double) * nc, hipMemcpyDeviceToHost, h->stream), "copy dt");
        hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        double mn = DBL_MAX;
        for (double v : cdt) mn = std::min(mn, v);
        h->dt = gas->dt_override > 0.0 ? gas->dt_override : gas->cfl * mn;
        if (!(h->dt > 0.0) || h->dt >= DBL_MAX) throw Fail{UGKS_ERR_ARG, "could not form a time step"};
        P.dt = h->dt;

        // pinned status copies for asynchronous and batched steps, and this
        // device's scratch of the allocation-free batched step
        ensure_async(h);
        void *scr = nullptr;
        hip_check(static_scratch(&scr), "device scratch address");
        hip_check(launch_init(P, prim_d, h->f[0], h->stream), "k_init launch");
        hip_check(launch_moments(P, h->f[0], h->stream), "k_moments launch");
        hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        (void)hipFree(prim_d);
        prim_d = nullptr;
        h->bytes -= sizeof(double) * nc * (D + 2);
    } catch (const Fail &e) {
        if (prim_d) (void)hipFree(prim_d);
        release(h);
        delete h;
        return fail(nullptr, e);
    } catch (const std::exception &e) {
        if (prim_d) (void)hipFree(prim_d);
        release(h);
        delete h;
        return fail(nullptr, Fail{UGKS_ERR_ALLOC, std::string("host: ") + e.what()});
    }
    *out = h;
    return UGKS_OK;
}

namespace {
// one step's sweep: into the other buffer (then it becomes the current one),
// or in place
void sweep(ugks_t *h)
{
    if (h->mem_mode == UGKS_MEM_IN_PLACE && h->push) {
        hip_check(launch_push_inplace(h->P, h->f[0], h->colour_cells, h->colour_off.data(),
                                      (int)h->colour_off.size() - 1, h->wall_cells, h->n_wall_cells, h->stream),
                  "in-place push sweep launch");
        h->last_push = 1;
    } else if (h->mem_mode == UGKS_MEM_IN_PLACE) {
        hip_check(launch_sweep_inplace(h->P, h->f[0], h->n_wallf > 0, h->stream), "in-place sweep launch");
    } else if (h->push) {
        hip_check(launch_push_step(h->P, h->f[h->cur], h->f[1 - h->cur], !h->base_ok, h->colour_cells,
                                   h->colour_off.data(), (int)h->colour_off.size() - 1, h->wall_cells, h->n_wall_cells,
                                   h->stream),
                  "push sweep launch");
        h->base_ok = 1;
        h->last_push = 1;
    } else {
        hip_check(launch_sweep(h->P, h->f[h->cur], h->f[1 - h->cur], h->stream), "sweep launch");
        h->cur ^= 1;
    }
}
}  // namespace

extern "C" int ugks_step(ugks_t *h, int nsteps, double *residual_out)
{
    if (!h) return UGKS_ERR_ARG;
    if (nsteps < 0) return fail(h, Fail{UGKS_ERR_ARG, "nsteps < 0"});
    try {
        if (h->profiling && h->ev.size() < (size_t)3 * nsteps) {
            size_t old = h->ev.size();
            h->ev.resize((size_t)3 * nsteps);
            for (size_t e = old; e < h->ev.size(); ++e) hip_check(hipEventCreate(&h->ev[e]), "hipEventCreate");
        }
        for (int s = 0; s < nsteps; ++s) {
            if (h->profiling) hip_check(hipEventRecord(h->ev[3 * s], h->stream), "hipEventRecord");
            hip_check(launch_prologue(h->P, h->stream), "prologue launch");
            if (h->profiling) hip_check(hipEventRecord(h->ev[3 * s + 1], h->stream), "hipEventRecord");
            sweep(h);
            if (h->profiling) hip_check(hipEventRecord(h->ev[3 * s + 2], h->stream), "hipEventRecord");
            h->nstep++;
            h->stepped = 1;
        }
        int err[2];
        hip_check(hipMemcpyAsync(err, h->err, sizeof(err), hipMemcpyDeviceToHost, h->stream), "copy error flag");
        if (residual_out && nsteps > 0) {
            hip_check(launch_residual(h->P, h->res, h->stream), "residual launch");
            hip_check(hipMemcpyAsync(residual_out, h->res, sizeof(double) * (h->dim + 2), hipMemcpyDeviceToHost, h->stream),
                      "copy residual");
        }
        hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        if (h->profiling)
            for (int s = 0; s < nsteps; ++s) {
                float a = 0.f, b = 0.f;
                hip_check(hipEventElapsedTime(&a, h->ev[3 * s], h->ev[3 * s + 1]), "hipEventElapsedTime");
                hip_check(hipEventElapsedTime(&b, h->ev[3 * s + 1], h->ev[3 * s + 2]), "hipEventElapsedTime");
                h->prof_ms[0] += b;
                h->prof_ms[1] += a;
                h->prof_n++;
            }
        if (err[0]) return fail(h, Fail{UGKS_ERR_NONPHYSICAL, nonphysical_message(h, err[1])});
    } catch (const Fail &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, Fail{UGKS_ERR_ALLOC, std::string("host: ") + e.what()});
    }
    return UGKS_OK;
}

extern "C" int ugks_step_async(ugks_t *h, int nsteps)
{
    if (!h) return UGKS_ERR_ARG;
    if (nsteps <= 0) return fail(h, Fail{UGKS_ERR_ARG, "nsteps must be positive"});
    if (h->pending) return fail(h, Fail{UGKS_ERR_STATE, "previous asynchronous steps not yet polled to completion"});
    try {
        ensure_async(h);
        for (int s = 0; s < nsteps; ++s) {
            hip_check(launch_prologue(h->P, h->stream), "prologue launch");
            sweep(h);
            h->nstep++;
            h->stepped = 1;
        }
        hip_check(launch_residual(h->P, h->res, h->stream), "residual launch");
        finish_async(h);
    } catch (const Fail &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, Fail{UGKS_ERR_ALLOC, std::string("host: ") + e.what()});
    }
    return UGKS_OK;
}

extern "C" int ugks_poll(ugks_t *h, int *done, double *residual_out)
{
    if (!h || !done) return UGKS_ERR_ARG;
    if (!h->pending) {
        *done = 1;
        return UGKS_OK;
    }
    const hipError_t q = hipEventQuery(h->done_ev);
    if (q == hipErrorNotReady) {
        *done = 0;
        return UGKS_OK;
    }
    h->pending = 0;
    *done = 1;
    if (q != hipSuccess) return fail(h, Fail{UGKS_ERR_HIP, std::string("hipEventQuery: ") + hipGetErrorString(q)});
    if (residual_out)
        for (int m = 0; m < h->dim + 2; ++m) residual_out[m] = h->h_res[m];
    if (h->h_err[0])
        return fail(h, Fail{UGKS_ERR_NONPHYSICAL, nonphysical_message(h, h->h_err[1])});
    return UGKS_OK;
}

extern "C" size_t ugks_footprint_estimate(const ugks_mesh_t *mesh, const ugks_vgrid_t *vgrid, const ugks_gas_t *gas)
{
    if (!mesh || !vgrid || !gas || (mesh->dim != 2 && mesh->dim != 3) || vgrid->dim != mesh->dim || !vgrid->u)
        return 0;
    int n1d[3];
    std::vector<double> axes;
    std::vector<int> kidx;
    size_t ntab = 0;
    if (detect_tensor(mesh->dim, vgrid->n_vel, vgrid->u, n1d, axes, kidx) &&
        (size_t)(Dim<3>::MF + 1) * axes.size() * sizeof(double) <= 48 * 1024)
        ntab = axes.size();
    size_t nwallf = 0;
    if (mesh->face_bc)
        for (int f = 0; f < mesh->n_faces; ++f) nwallf += mesh->face_bc[f] == UGKS_BC_WALL;
    return plan_bytes(mesh->dim, mesh->n_cells, mesh->n_faces, vgrid->n_vel, gas->n_bc, gas->fstore, ntab, nwallf,
                      gas->mem_mode, gas->chunk, uses_push(mesh->dim, gas));
}

extern "C" int ugks_macros(ugks_t *h, double *W_out, double *q_out)
{
    if (!h) return UGKS_ERR_ARG;
    try {
        const size_t nc = h->nc, NW = h->dim + 2, D = h->dim;
        std::vector<double> W(W_out ? nc * NW : 0), q(q_out ? nc * D : 0);
        if (W_out) hip_check(hipMemcpyAsync(W.data(), h->W, sizeof(double) * W.size(), hipMemcpyDeviceToHost, h->stream), "copy W");
        if (q_out) hip_check(hipMemcpyAsync(q.data(), h->q, sizeof(double) * q.size(), hipMemcpyDeviceToHost, h->stream), "copy q");
        hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        for (size_t i = 0; i < nc; ++i) {
            const size_t c = h->cell_of[i];
            if (W_out) std::copy(&W[i * NW], &W[i * NW] + NW, W_out + c * NW);
            if (q_out) std::copy(&q[i * D], &q[i * D] + D, q_out + c * D);
        }
    } catch (const Fail &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, Fail{UGKS_ERR_ALLOC, std::string("host: ") + e.what()});
    }
    return UGKS_OK;
}

extern "C" int ugks_get_f(ugks_t *h, double *f_out)
{
    if (!h || !f_out) return UGKS_ERR_ARG;
    try {
        const size_t nv = h->nv, rows = (size_t)h->nc * h->ncomp, n = rows * nv;
        std::vector<double> tmp(n);
        if (h->fstore == UGKS_F64) {
            hip_check(hipMemcpyAsync(tmp.data(), h->f[h->cur], sizeof(double) * n, hipMemcpyDeviceToHost, h->stream), "copy f");
            hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        } else if (h->fstore == UGKS_F32) {
            std::vector<float> t32(n);
            hip_check(hipMemcpyAsync(t32.data(), h->f[h->cur], sizeof(float) * n, hipMemcpyDeviceToHost, h->stream), "copy f");
            hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
            for (size_t i = 0; i < n; ++i) tmp[i] = t32[i];
        } else {
            std::vector<uint16_t> t16(n);
            hip_check(hipMemcpyAsync(t16.data(), h->f[h->cur], 2 * n, hipMemcpyDeviceToHost, h->stream), "copy f");
            hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
            for (size_t i = 0; i < n; ++i) tmp[i] = double_of_bf16(t16[i]);
        }
        const size_t nk = h->ncomp;
        for (size_t r = 0; r < rows; ++r) {
            double *dst = f_out + ((size_t)h->cell_of[r / nk] * nk + r % nk) * nv;
            for (size_t k = 0; k < nv; ++k) dst[h->perm[k]] = tmp[r * nv + k];
        }
    } catch (const Fail &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, Fail{UGKS_ERR_ALLOC, std::string("host: ") + e.what()});
    }
    return UGKS_OK;
}

extern "C" int ugks_set_f(ugks_t *h, const double *f_in)
{
    if (!h || !f_in) return UGKS_ERR_ARG;
    if (h->pending) return fail(h, Fail{UGKS_ERR_STATE, "asynchronous steps not yet polled to completion"});
    h->stepped = 0;
    h->base_ok = 0;
    try {
        const size_t nv = h->nv, rows = (size_t)h->nc * h->ncomp, n = rows * nv;
        std::vector<double> tmp(n);
        const size_t nk = h->ncomp;
        const int err0[2] = {0, 0x7fffffff};  // a new state: clear the non-physical flag
        upload(h->err, err0, sizeof(err0), h->stream);
        for (size_t r = 0; r < rows; ++r) {
            const double *src = f_in + ((size_t)h->cell_of[r / nk] * nk + r % nk) * nv;
            for (size_t k = 0; k < nv; ++k) tmp[r * nv + k] = src[h->perm[k]];
        }
        if (h->fstore == UGKS_F64) {
            upload(h->f[h->cur], tmp.data(), sizeof(double) * n, h->stream);
            hip_check(launch_moments(h->P, h->f[h->cur], h->stream), "k_moments launch");
            hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        } else if (h->fstore == UGKS_F32) {
            std::vector<float> t32(n);
            for (size_t i = 0; i < n; ++i) t32[i] = (float)tmp[i];
            upload(h->f[h->cur], t32.data(), sizeof(float) * n, h->stream);
            hip_check(launch_moments(h->P, h->f[h->cur], h->stream), "k_moments launch");
            hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        } else {
            std::vector<uint16_t> t16(n);
            for (size_t i = 0; i < n; ++i) t16[i] = bf16_of(tmp[i]);
            upload(h->f[h->cur], t16.data(), 2 * n, h->stream);
            hip_check(launch_moments(h->P, h->f[h->cur], h->stream), "k_moments launch");
            hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        }
    } catch (const Fail &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, Fail{UGKS_ERR_ALLOC, std::string("host: ") + e.what()});
    }
    return UGKS_OK;
}

// ------------------------------------------------------------------------
// checkpoint: the exact state of a handle (W, q, f in its storage precision
// and the library's order, step count), restorable into a handle created
// from the same inputs
// ------------------------------------------------------------------------
namespace {
struct StateHeader {
    char magic[8];  // "UGKSST01"
    int dim, nc, nv, ncomp, fstore, pad;
    long nstep;
    unsigned long long order_hash;  // of the library's cell and velocity orders
};

unsigned long long order_hash(const ugks_t *h)
{
    unsigned long long x = 1469598103934665603ull;  // FNV-1a over both permutations
    auto mix = [&](int v) {
        for (int b = 0; b < 4; ++b) {
            x ^= (unsigned long long)((v >> (8 * b)) & 0xff);
            x *= 1099511628211ull;
        }
    };
    for (int v : h->cell_of) mix(v);
    for (int v : h->perm) mix(v);
    return x;
}

size_t state_bytes(const ugks_t *h)
{
    const size_t nc = h->nc, NW = h->dim + 2;
    return sizeof(StateHeader) + sizeof(double) * nc * (NW + h->dim) + nc * h->ncomp * h->nv * fvalue_bytes(h->fstore);
}
}  // namespace

extern "C" size_t ugks_state_bytes(const ugks_t *h) { return h ? state_bytes(h) : 0; }

extern "C" int ugks_get_state(ugks_t *h, void *buf, size_t bytes)
{
    if (!h || !buf) return UGKS_ERR_ARG;
    if (bytes < state_bytes(h)) return fail(h, Fail{UGKS_ERR_ARG, "state buffer too small (see ugks_state_bytes)"});
    if (h->pending) return fail(h, Fail{UGKS_ERR_STATE, "asynchronous steps not yet polled to completion"});
    try {
        StateHeader hd{};
        std::memcpy(hd.magic, "UGKSST01", 8);
        hd.dim = h->dim;
        hd.nc = h->nc;
        hd.nv = h->nv;
        hd.ncomp = h->ncomp;
        hd.fstore = h->fstore;
        hd.nstep = h->nstep;
        hd.order_hash = order_hash(h);
        char *p = static_cast<char *>(buf);
        std::memcpy(p, &hd, sizeof(hd));
        p += sizeof(hd);
        const size_t nW = sizeof(double) * h->nc * (h->dim + 2), nq = sizeof(double) * h->nc * h->dim;
        const size_t nf = (size_t)h->nc * h->ncomp * h->nv * fvalue_bytes(h->fstore);
        hip_check(hipMemcpyAsync(p, h->W, nW, hipMemcpyDeviceToHost, h->stream), "copy W");
        hip_check(hipMemcpyAsync(p + nW, h->q, nq, hipMemcpyDeviceToHost, h->stream), "copy q");
        hip_check(hipMemcpyAsync(p + nW + nq, h->f[h->cur], nf, hipMemcpyDeviceToHost, h->stream), "copy f");
        hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    } catch (const Fail &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, Fail{UGKS_ERR_ALLOC, std::string("host: ") + e.what()});
    }
    return UGKS_OK;
}

extern "C" int ugks_set_state(ugks_t *h, const void *buf, size_t bytes)
{
    if (!h || !buf) return UGKS_ERR_ARG;
    if (h->pending) return fail(h, Fail{UGKS_ERR_STATE, "asynchronous steps not yet polled to completion"});
    if (bytes < sizeof(StateHeader)) return fail(h, Fail{UGKS_ERR_ARG, "state buffer too small"});
    StateHeader hd;
    std::memcpy(&hd, buf, sizeof(hd));
    if (std::memcmp(hd.magic, "UGKSST01", 8) != 0) return fail(h, Fail{UGKS_ERR_ARG, "not a UGKS state"});
    if (hd.dim != h->dim || hd.nc != h->nc || hd.nv != h->nv || hd.ncomp != h->ncomp || hd.fstore != h->fstore ||
        hd.order_hash != order_hash(h))
        return fail(h, Fail{UGKS_ERR_ARG, "state of a different case (sizes, storage or orders differ)"});
    if (bytes < state_bytes(h)) return fail(h, Fail{UGKS_ERR_ARG, "state buffer truncated"});
    try {
        const char *p = static_cast<const char *>(buf) + sizeof(hd);
        const size_t nW = sizeof(double) * h->nc * (h->dim + 2), nq = sizeof(double) * h->nc * h->dim;
        const size_t nf = (size_t)h->nc * h->ncomp * h->nv * fvalue_bytes(h->fstore);
        upload(h->W, p, nW, h->stream);
        upload(h->q, p + nW, nq, h->stream);
        upload(h->f[h->cur], p + nW + nq, nf, h->stream);
        const int err0[2] = {0, 0x7fffffff};
        upload(h->err, err0, sizeof(err0), h->stream);
        hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        h->nstep = hd.nstep;
        h->stepped = 0;
        h->base_ok = 0;
    } catch (const Fail &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, Fail{UGKS_ERR_ALLOC, std::string("host: ") + e.what()});
    }
    return UGKS_OK;
}

extern "C" int ugks_n_wall_faces(const ugks_t *h) { return h ? h->n_wallf : 0; }

extern "C" int ugks_wall_flux(ugks_t *h, double *out)
{
    if (!h || !out) return UGKS_ERR_ARG;
    if (h->pending) return fail(h, Fail{UGKS_ERR_STATE, "asynchronous steps not yet polled to completion"});
    if (!h->stepped) return fail(h, Fail{UGKS_ERR_STATE, "no step since creation or ugks_set_f"});
    if (h->mem_mode == UGKS_MEM_IN_PLACE && !h->last_push)
        return fail(h, Fail{UGKS_ERR_STATE, "an in-place gather handle keeps no copy of the f that started the step"});
    try {
        if (h->n_wallf) {
            if (!h->last_push)  // a push step recorded its wall flux; else recompute it from the f that started it
                hip_check(launch_wall_flux(h->P, h->f[1 - h->cur], h->wallf, h->n_wallf, h->wallF, h->stream),
                          "wall flux launch");
            hip_check(hipMemcpyAsync(out, h->wallF, sizeof(double) * h->n_wallf * (h->dim + 2), hipMemcpyDeviceToHost,
                                     h->stream), "copy wall flux");
            hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        }
    } catch (const Fail &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, Fail{UGKS_ERR_ALLOC, std::string("host: ") + e.what()});
    }
    return UGKS_OK;
}

extern "C" int ugks_surface(ugks_t *h, double rho_inf, double u_inf, double *out)
{
    if (!h || !out) return UGKS_ERR_ARG;
    if (!(rho_inf > 0.0) || !(u_inf > 0.0) || !std::isfinite(rho_inf) || !std::isfinite(u_inf))
        return fail(h, Fail{UGKS_ERR_ARG, "rho_inf and u_inf must be positive and finite"});
    if (h->pending) return fail(h, Fail{UGKS_ERR_STATE, "asynchronous steps not yet polled to completion"});
    if (!h->stepped) return fail(h, Fail{UGKS_ERR_STATE, "no step since creation or ugks_set_f"});
    if (h->mem_mode == UGKS_MEM_IN_PLACE && !h->last_push)
        return fail(h, Fail{UGKS_ERR_STATE, "an in-place gather handle keeps no copy of the f that started the step"});
    try {
        if (h->n_wallf) {
            if (!h->last_push)
                hip_check(launch_wall_flux(h->P, h->f[1 - h->cur], h->wallf, h->n_wallf, h->wallF, h->stream),
                          "wall flux launch");
            hip_check(launch_surface(h->P, h->wallf, h->wallF, h->n_wallf, rho_inf, u_inf, h->surf, h->stream),
                      "surface launch");
            hip_check(hipMemcpyAsync(out, h->surf, sizeof(double) * h->n_wallf * 6, hipMemcpyDeviceToHost, h->stream),
                      "copy surface quantities");
            hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        }
    } catch (const Fail &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, Fail{UGKS_ERR_ALLOC, std::string("host: ") + e.what()});
    }
    return UGKS_OK;
}

extern "C" int ugks_velocity_order(const ugks_t *h, int *perm_out)
{
    if (!h || !perm_out) return UGKS_ERR_ARG;
    std::copy(h->perm.begin(), h->perm.end(), perm_out);
    return UGKS_OK;
}

extern "C" int ugks_cell_order(const ugks_t *h, int *perm_out)
{
    if (!h || !perm_out) return UGKS_ERR_ARG;
    std::copy(h->cell_of.begin(), h->cell_of.end(), perm_out);
    return UGKS_OK;
}

extern "C" int ugks_profile(ugks_t *h, int enable)
{
    if (!h) return UGKS_ERR_ARG;
    h->profiling = enable ? 1 : 0;
    h->prof_ms[0] = h->prof_ms[1] = 0.0;
    h->prof_n = 0;
    return UGKS_OK;
}

extern "C" int ugks_profile_read(const ugks_t *h, double *ms_out, long *launches)
{
    if (!h || !ms_out) return UGKS_ERR_ARG;
    ms_out[0] = h->prof_ms[0];
    ms_out[1] = h->prof_ms[1];
    if (launches) *launches = h->prof_n;
    return UGKS_OK;
}

extern "C" double ugks_dt(const ugks_t *h) { return h ? h->dt : -1.0; }
extern "C" int ugks_n_comp(const ugks_t *h) { return h ? h->ncomp : 0; }
extern "C" long ugks_step_count(const ugks_t *h) { return h ? h->nstep : -1; }
extern "C" size_t ugks_footprint_bytes(const ugks_t *h) { return h ? h->bytes : 0; }
extern "C" int ugks_sweep_kind(const ugks_t *h)
{
    if (!h) return -1;
    return h->push ? (h->unordered ? UGKS_SWEEP_PUSH_UNORDERED : UGKS_SWEEP_PUSH) : UGKS_SWEEP_GATHER;
}

extern "C" int ugks_sweep_colours(const ugks_t *h)
{
    if (!h) return -1;
    return h->push ? (int)h->colour_off.size() - 1 : 0;
}

extern "C" int ugks_is_tensor_grid(const ugks_t *h) { return h ? h->tensor : 0; }
extern "C" const void *ugks_device_f(const ugks_t *h) { return h ? h->f[h->cur] : nullptr; }

extern "C" void ugks_destroy(ugks_t *h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    release(h);
    delete h;
}

extern "C" const char *ugks_last_error(const ugks_t *h) { return h ? h->msg.c_str() : g_create_error.c_str(); }

// ------------------------------------------------------------------------
// batched stepping of several cases by the same launches
// ------------------------------------------------------------------------
struct ugks_batch {
    hipStream_t stream = nullptr;
    int max_cases = 0;
    BatchItem *items = nullptr;  // device [max_cases]
    int *off = nullptr;          // device: prologue offsets [2][max + 1], sweep offsets up to [max + max]
    BatchItem *h_items = nullptr;  // pinned staging of the same
    int *h_off = nullptr;
    hipEvent_t up_ev = nullptr;    // recorded after the last uploads
    int uploaded = 0;
    std::string msg;
};

extern "C" int ugks_batch_create(int max_cases, void *stream, ugks_batch_t **out)
{
    if (!out || max_cases <= 0) return UGKS_ERR_ARG;
    *out = nullptr;
    ugks_batch_t *b = new (std::nothrow) ugks_batch_t();
    if (!b) return UGKS_ERR_ALLOC;
    b->stream = static_cast<hipStream_t>(stream);
    b->max_cases = max_cases;
    const size_t noff = 4 * (size_t)max_cases + 3;
    if (hipMalloc((void **)&b->items, sizeof(BatchItem) * max_cases) != hipSuccess ||
        hipMalloc((void **)&b->off, sizeof(int) * noff) != hipSuccess ||
        hipHostMalloc((void **)&b->h_items, sizeof(BatchItem) * max_cases, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&b->h_off, sizeof(int) * noff, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->up_ev, hipEventDisableTiming) != hipSuccess) {
        if (b->items) (void)hipFree(b->items);
        if (b->off) (void)hipFree(b->off);
        if (b->h_items) (void)hipHostFree(b->h_items);
        if (b->h_off) (void)hipHostFree(b->h_off);
        delete b;
        g_create_error = "allocation of the batch descriptors failed";
        return UGKS_ERR_ALLOC;
    }
    *out = b;
    return UGKS_OK;
}

namespace {
// one group of a batched sweep: cases sharing the sweep's instantiation
struct SweepGroup {
    int first, count, grid;
    size_t lds;
    long key;
    size_t off_at;  // its offset table inside off[]
};
constexpr int kMaxSweepGroups = 12;  // storage (3) x per-axis tables (2) x stage-1 place (2)

// Checks of a batch: NULL, stream, dimension, pending steps, memory mode,
// BF16 push handles (whose two buffers differ in size), duplicates.  0 or
// an error code, with the reason in why (static text).
int batch_check(ugks_t *const *hs, int n, hipStream_t stream, const char **why)
{
    const int D = hs[0] ? hs[0]->dim : 0;
    for (int c = 0; c < n; ++c) {
        const ugks_t *h = hs[c];
        if (!h) return *why = "NULL handle in the batch", UGKS_ERR_ARG;
        if (h->stream != stream) return *why = "every handle of a batch must use the batch's stream", UGKS_ERR_ARG;
        if (h->dim != D) return *why = "cases of one batch must have the same dimension", UGKS_ERR_ARG;
        if (h->pending) return *why = "a handle still has asynchronous steps outstanding", UGKS_ERR_STATE;
        if (h->mem_mode == UGKS_MEM_IN_PLACE) return *why = "in-place handles cannot be batched", UGKS_ERR_ARG;
        if (h->push && h->fstore == UGKS_BF16)
            return *why = "BF16 handles with the push sweep cannot be batched (FP32 stage-1 sums)", UGKS_ERR_ARG;
        if (!h->h_err) return *why = "handle without its pinned status copies", UGKS_ERR_STATE;
        for (int e = 0; e < c; ++e)
            if (hs[e] == h) return *why = "a handle appears twice in the batch", UGKS_ERR_ARG;
    }
    return 0;
}

// Host layout of one batched step of hs[0..n): the descriptors items[0..n)
// in sweep-group order, the offset tables off[0 .. 4n+3) (prologue: cell
// gradients [n+1], face equilibria [n+1]; then one sweep table per group),
// and the sweep groups.  order, key and lds are work arrays of n entries.
// Nothing is allocated.
int batch_layout(ugks_t *const *hs, int n, BatchItem *items, int *off, int *order, long *key, size_t *lds,
                 SweepGroup *groups)
{
    for (int c = 0; c < n; ++c) {
        bool s1l = false;
        lds[c] = sweep_lds_bytes(hs[c]->P, &s1l);
        key[c] = hs[c]->fstore * 4 + (hs[c]->P.ntab > 0 ? 2 : 0) + (s1l ? 1 : 0);
        order[c] = c;
    }
    // stable insertion sort by key (a handful of cases)
    for (int a = 1; a < n; ++a) {
        const int v = order[a];
        int b = a;
        while (b > 0 && key[order[b - 1]] > key[v]) {
            order[b] = order[b - 1];
            --b;
        }
        order[b] = v;
    }
    std::fill(off, off + 4 * (size_t)n + 3, 0);
    int *og = off, *of = og + (n + 1), *os = of + (n + 1);
    for (int j = 0; j < n; ++j) {
        const ugks_t *h = hs[order[j]];
        items[j].p = h->P;
        items[j].f[0] = h->f[0];
        items[j].f[1] = h->f[1];
        items[j].res = h->res;
        items[j].cur = h->cur;
        og[j + 1] = og[j] + (h->nc + 255) / 256;
        of[j + 1] = of[j] + (h->nf + 127) / 128;
    }
    int ng = 0;
    size_t at = 0;
    for (int j = 0; j < n;) {
        int e = j;
        size_t mx = 0;
        while (e < n && key[order[e]] == key[order[j]]) mx = std::max(mx, lds[order[e++]]);
        SweepGroup &g = groups[ng++];
        g = SweepGroup{j, e - j, 0, mx, key[order[j]], (size_t)(os - off) + at};
        int *t = os + at;
        t[0] = 0;
        for (int q = 0; q < g.count; ++q) t[q + 1] = t[q] + sweep_grid(hs[order[j + q]]->nc);
        g.grid = t[g.count];
        at += g.count + 1;
        j = e;
    }
    return ng;
}

// The launches of nsteps batched steps from descriptors already on the
// device, then each handle's bookkeeping and its status copies.
hipError_t batch_launch(ugks_t *const *hs, int n, int nsteps, const BatchItem *d_items, const int *d_off,
                        const int *h_off, const SweepGroup *groups, int ng, hipStream_t s)
{
    const int D = hs[0]->dim;
    hipError_t e = hipSuccess;
    for (int st = 0; st < nsteps && e == hipSuccess; ++st) {
        e = launch_batch_prologue(d_items, n, d_off, h_off[n], d_off + (n + 1), h_off[2 * n + 1], D, s);
        for (int g = 0; g < ng && e == hipSuccess; ++g)
            e = launch_batch_sweep(d_items + groups[g].first, groups[g].count, d_off + groups[g].off_at, groups[g].grid,
                                   st, D, (int)(groups[g].key / 4), (groups[g].key & 2) != 0,
                                   (groups[g].key & 1) != 0, groups[g].lds, s);
    }
    if (e == hipSuccess) e = launch_batch_residual(d_items, n, D, s);
    for (int c = 0; c < n && e == hipSuccess; ++c) {
        ugks_t *h = hs[c];
        h->cur ^= (nsteps & 1);
        h->nstep += nsteps;
        h->stepped = 1;
        h->base_ok = 0;  // gather steps: the second buffer no longer holds the base
        h->last_push = 0;
        e = hipMemcpyAsync(h->h_err, h->err, 2 * sizeof(int), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->h_res, h->res, (h->dim + 2) * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipEventRecord(h->done_ev, h->stream);
        if (e == hipSuccess) h->pending = 1;
    }
    return e;
}

}  // namespace

extern "C" int ugks_batch_step(ugks_batch_t *b, ugks_t *const *hs, int n, int nsteps)
{
    if (!b) return UGKS_ERR_ARG;
    auto bad = [&](int code, const std::string &m) {
        b->msg = m;
        return code;
    };
    if (!hs || n <= 0 || n > b->max_cases) return bad(UGKS_ERR_ARG, "n must be in 1..max_cases");
    if (nsteps <= 0) return bad(UGKS_ERR_ARG, "nsteps must be positive");
    const char *why = "";
    if (const int code = batch_check(hs, n, b->stream, &why)) return bad(code, why);
    try {
        std::vector<int> order(n);
        std::vector<long> key(n);
        std::vector<size_t> lds(n);
        SweepGroup groups[kMaxSweepGroups];
        // the staging buffers are reused: wait until the previous uploads have left them
        if (b->uploaded) hip_check(hipEventSynchronize(b->up_ev), "hipEventSynchronize");
        const int ng = batch_layout(hs, n, b->h_items, b->h_off, order.data(), key.data(), lds.data(), groups);
        upload(b->items, b->h_items, sizeof(BatchItem) * n, b->stream);
        upload(b->off, b->h_off, sizeof(int) * (4 * (size_t)n + 3), b->stream);
        hip_check(hipEventRecord(b->up_ev, b->stream), "hipEventRecord");
        b->uploaded = 1;
        hip_check(batch_launch(hs, n, nsteps, b->items, b->off, b->h_off, groups, ng, b->stream), "batched step");
    } catch (const Fail &e) {
        return bad(e.code, e.msg);
    } catch (const std::exception &e) {
        return bad(UGKS_ERR_ALLOC, std::string("host: ") + e.what());
    }
    return UGKS_OK;
}

extern "C" int ugks_batch_step_static(ugks_t *const *hs, int n, int nsteps, void *stream)
{
    auto bad = [](int code, const char *m) {
        std::snprintf(g_static_batch_error, sizeof(g_static_batch_error), "%s", m);
        return code;
    };
    if (!hs || n <= 0) return bad(UGKS_ERR_ARG, "hs must hold at least one handle");
    if (n > UGKS_STATIC_BATCH_MAX) return bad(UGKS_ERR_ARG, "at most UGKS_STATIC_BATCH_MAX (64) cases per call");
    if (nsteps <= 0) return bad(UGKS_ERR_ARG, "nsteps must be positive");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const char *why = "";
    if (const int code = batch_check(hs, n, s, &why)) return bad(code, why);
    void *base = nullptr;
    if (static_scratch(&base) != hipSuccess) return bad(UGKS_ERR_HIP, "device scratch address lookup failed");
    BatchItem *d_items = static_cast<BatchItem *>(base);
    int *d_off = reinterpret_cast<int *>(static_cast<unsigned char *>(base) + kStaticItemsBytes);
    // host layout on the stack: nothing is allocated
    BatchItem items[UGKS_STATIC_BATCH_MAX];
    int off[4 * UGKS_STATIC_BATCH_MAX + 3];
    int order[UGKS_STATIC_BATCH_MAX];
    long key[UGKS_STATIC_BATCH_MAX];
    size_t lds[UGKS_STATIC_BATCH_MAX];
    SweepGroup groups[kMaxSweepGroups];
    const int ng = batch_layout(hs, n, items, off, order, key, lds, groups);
    // the layout leaves the stack before returning: copy it and wait for the copy
    hipError_t e = hipMemcpyAsync(d_items, items, sizeof(BatchItem) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_off, off, sizeof(int) * (4 * (size_t)n + 3), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = batch_launch(hs, n, nsteps, d_items, d_off, off, groups, ng, s);
    if (e != hipSuccess) return bad(UGKS_ERR_HIP, hipGetErrorString(e));
    g_static_batch_error[0] = 0;
    return UGKS_OK;
}

extern "C" const char *ugks_batch_last_error(const ugks_batch_t *b)
{
    if (b) return b->msg.c_str();
    return g_static_batch_error[0] ? g_static_batch_error : g_create_error.c_str();
}

extern "C" void ugks_batch_destroy(ugks_batch_t *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    (void)hipFree(b->items);
    (void)hipFree(b->off);
    (void)hipHostFree(b->h_items);
    (void)hipHostFree(b->h_off);
    (void)hipEventDestroy(b->up_ev);
    delete b;
}
