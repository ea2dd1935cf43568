// ugks_internal.h -- device data layout and launch interface shared by the
// host library (ugks_api.cpp) and the gfx950 kernels (ugks_kernels.hip).
// Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace ugx {

// Faces per cell: 2D triangles/quads (<= 4), 3D tets/prisms/hexes (<= 6).
template <int D> struct Dim;
template <> struct Dim<2> {
    static constexpr int MF = 4;  // max faces per cell
    static constexpr int NC = 2;  // stored components: h, b
    static constexpr int M = 1;   // internal velocity components (xi)
    static constexpr int NW = 4;  // conservative variables
};
template <> struct Dim<3> {
    static constexpr int MF = 6;
    static constexpr int NC = 1;  // b is identically zero without internal components
    static constexpr int M = 0;
    static constexpr int NW = 5;
};

// Per-cell stencil record, read with wave-uniform (scalar) loads.
template <int D> struct alignas(16) CellGeo {
    static constexpr int MF = Dim<D>::MF;
    int nf;          // faces of the cell
    int face[MF];    // face index per slot
    int nb[MF];      // neighbour across the slot's face, -1 on a boundary
    int back[MF];    // slot index of this face in the neighbour's record
    int side[MF];    // 0: the cell is the face's left cell, 1: right
    double inv_vol;  // 1 / |Omega_i|
    double eps2;     // Venkatakrishnan epsilon^2
    double dvec[MF][D];  // centroid -> face centroid, in this cell's frame
    double lsq[MF][D];   // least-squares weights: grad = sum_j lsq_j (f_j - f_i)
    double nb_inv_vol[MF];  // 1 / |Omega_n| of the neighbour across each slot (0 on a boundary)
};

template <int D> struct alignas(16) FaceGeo {
    int l, r, bc, bcid;
    double n[D];   // unit normal, left -> right
    double area;
    double dl[D];  // left centroid -> face centroid
    double dr[D];  // right centroid (its periodic image) -> face centroid
};

// Interface equilibrium (Algorithm 1's third step).  For boundary faces only
// (rho, U, lam) and pref are used: ghost Maxwellian (inflow), wall Maxwellian
// with unit density (wall).
template <int D> struct alignas(16) FaceEq {
    static constexpr int NW = D + 2;
    double rho, U[D], lam;
    double pref;          // rho (lam/pi)^{D/2}
    double shk;           // 4 (1 - Pr) lam^2 / (5 rho)
    double bh;            // M / (2 lam): B = bh H
    double x4;            // M (M + 2) / (4 lam^2): int xi^4 g dxi = x4 H
    double a[D][NW];      // spatial slopes of g0
    double A[NW];         // time slope of g0
    double q[D];          // interface heat flux
    double c[5];          // time integrals of c1..c5 over the step
    // the step and (dt / 2) dt for the free-transport and boundary fluxes; the
    // sweep reads them with the face's other scalars, as the kernel argument
    // kept live across the velocity loop costs scalar-register spill reloads
    double dt, hdt2;
};

struct Params {
    int dim, fstore;
    int nc, nf, nv;
    double dt, Pr, omega, mu_ref;
    int limiter;
    // device arrays
    const void *cgeo, *fgeo;
    void *feq;
    const double *u;   // [dim][nv] (structure of arrays)
    const double *w;   // [nv]
    // Cartesian velocity grids: 1D axes [nx | ny | nz] and per-velocity axis
    // indices packed as a | b << 10 | c << 20; ntab = nx + ny + nz, 0 otherwise
    const double *u1d;
    const int *kidx;
    int n1d[3];
    int ntab;
    const double *bc_prim;  // [n_bc][dim+2]
    double *W, *q;     // [nc][dim+2], [nc][dim]
    double *gW;        // [nc][dim+2][dim] limited gradients of W
    double *dW2;       // [nc][dim+2] squared change of W in the last step
    int *err;          // [2]: flag, first bad cell
    // in-place mode (one f buffer): stage-1 values of the current velocity
    // chunk [cell][component][chunk], the moments of the net outflow of the
    // chunks swept so far, summed in chunk order [cell][dim+2], wall densities
    // [cell][MF]
    void *ring;
    int chunk, nchunk;
    double *mom_part, *rho_w;
    // push sweep: mom_part holds the moments of the stage-1 base [cell][dim+2];
    // wall ordinal of every face (-1 if not a wall) and the wall flux of the
    // last step per wall face [n_wall][dim+2] (per unit area and time)
    const int *wall_index;
    double *wflux;
    // push sweep with one f buffer: the stage-1 moments about U^n summed over
    // the chunks so far [cell][Shift<D>::N]
    double *mom_s;
};

// One case of a batched launch (several cases advanced by the same kernels):
// its parameters, its two f buffers and which one holds f when the batch
// starts, and where its residual goes.
struct BatchItem {
    Params p;
    const void *f[2];
    double *res;
    int cur;
};

// Allocation-free batched step: its descriptors (at most kStaticBatchMax
// cases) live in a fixed device array of kStaticScratchBytes, items first,
// then the offset tables (4 n + 3 ints).  static_scratch() gives the current
// device's copy of it (its address is looked up once per device).
constexpr int kStaticBatchMax = 64;
constexpr size_t kStaticItemsBytes = ((sizeof(BatchItem) * kStaticBatchMax + 255) / 256) * 256;
constexpr size_t kStaticScratchBytes = kStaticItemsBytes + sizeof(int) * (4 * kStaticBatchMax + 3);
hipError_t static_scratch(void **out);

// Dynamic LDS of the sweep for one case, and whether its stage-1 values
// stay in LDS (s1l).
size_t sweep_lds_bytes(const Params &p, bool *s1l);
// Batched launches over items[0..n): off_* are the per-case first workgroup
// (n + 1 entries, the last one the grid size) of each kernel's grid.
hipError_t launch_batch_prologue(const BatchItem *items, int n, const int *off_grad, int grid_grad,
                                 const int *off_face, int grid_face, int dim, hipStream_t s);
hipError_t launch_batch_sweep(const BatchItem *items, int n, const int *off, int grid, int step, int dim, int fstore,
                              bool tensor, bool s1l, size_t lds, hipStream_t s);
hipError_t launch_batch_residual(const BatchItem *items, int n, int dim, hipStream_t s);
// workgroups of the per-cell sweep grid for nc cells (a multiple of the XCD span)
int sweep_grid(int nc);

hipError_t launch_cfl(const Params &p, double *cell_dt, hipStream_t s);
hipError_t launch_init(const Params &p, const double *prim0, void *f, hipStream_t s);
hipError_t launch_moments(const Params &p, const void *f, hipStream_t s);
hipError_t launch_prologue(const Params &p, hipStream_t s);  // k_cell_grad + k_face_eq
hipError_t launch_sweep(const Params &p, const void *f_in, void *f_out, hipStream_t s);
// the push sweep of one step (FP64 or FP32 f): the stage-1 base of f into acc
// first when need_base, then the wall cells (wall densities into rho_w and
// the step's wall flux), then one launch per colour over cells[coff[c] ..
// coff[c+1]) (coff: host array of ncol + 1 offsets into the device list
// cells), then stage 2 into f and the next base into acc
hipError_t launch_push_step(const Params &p, void *f, void *acc, bool need_base, const int *cells, const int *coff,
                            int ncol, const int *wall_cells, int n_wall_cells, hipStream_t s);
// the push sweep with one f buffer (FP64 or FP32 f): the wall cells, then per
// velocity chunk the base into the ring, one launch per colour, the stage-1
// values back into f; then W^{n+1}, q^{n+1} and stage 2 in place
hipError_t launch_push_inplace(const Params &p, void *f, const int *cells, const int *coff, int ncol,
                               const int *wall_cells, int n_wall_cells, hipStream_t s);
// the in-place step's sweep: wall densities (if walls), one kernel per
// velocity chunk, the final kernel; f is read and updated in place
hipError_t launch_sweep_inplace(const Params &p, void *f, bool walls, hipStream_t s);
// L2 norm over cells of the last change of W: out[0..D+2) receives it and
// out[D+2 ..) holds residual_groups(nc) * (D+2) partial sums
constexpr int kResidualGroups = 256;
int residual_groups(int nc);
hipError_t launch_residual(const Params &p, double *out, hipStream_t s);
// macroscopic flux [n][dim+2] through the wall faces faces[0..n) in the step that started from f
hipError_t launch_wall_flux(const Params &p, const void *f, const int *faces, int n, double *out, hipStream_t s);
// surface quantities [n][6] (p_w, sigma_w, q_w, Cp, Ct, Ch) from the wall flux [n][dim+2]
hipError_t launch_surface(const Params &p, const int *faces, const double *flux, int n, double rho_inf, double u_inf,
                          double *out, hipStream_t s);

}  // namespace ugx
