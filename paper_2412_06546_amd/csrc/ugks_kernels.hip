// ugks_kernels.hip -- gfx950 kernels of the memory-saving UGKS time step.
//
// Reference: Zhang, Wei, Long, Xu, "An efficiency and memory-saving
// programming paradigm for the unified gas-kinetic scheme", arXiv:2412.06546.
//
// One step (Algorithm 1 of Section 3.2) on one stream:
//   k_cell_grad  per cell:  limited least-squares gradient of W (the
//                           macroscopic reconstruction)
//   k_face_eq    per face:  interface equilibrium g0, its space and time
//                           slopes, heat flux and time integrals
//   then the velocity loop and the updates after it, by one of two sweeps:
//   push sweep   (default)  each cell computes its own limited slope of f
//                once per velocity and, for every face the velocity leaves
//                through, the interface flux of Eq. fullSolution integrated
//                over the step, added with atomic adds into the stage-1 sums
//                (Eq. microS1) of both of the face's cells: k_push_wall (wall
//                densities), k_push_pf / k_push (per colour class of cells,
//                or one launch of all cells), then k_push_final_r /
//                k_push_final (W^{n+1}, q^{n+1}, stage 2 of Eq. microS2);
//   gather sweep k_sweep    per cell, one workgroup owning the cell's whole
//                velocity slab: for every velocity the limited slope of f is
//                rebuilt in registers (own cell, and upwind neighbours when
//                the neighbour is upwind), the stage-1 value is kept in
//                registers, the wall density is reduced over velocities,
//                W^{n+1} and q^{n+1} come from workgroup reductions of the
//                same registers, and stage 2 is applied before the single
//                store.
// f is stored [cell][component][velocity]; lanes run over velocities, so a
// wavefront reads 64 consecutive velocities of one cell (coalesced) and all
// geometry and face data are wave-uniform (scalar loads).  f^n and the
// stage-1 sums (push) or f^{n+1} (gather) are in two buffers, or one buffer
// and a ring of one velocity chunk in place: no slope or residual of f ever
// reaches memory.
#include "ugks_internal.h"

#include <algorithm>
#include <mutex>

#include <cfloat>
#include <cmath>

namespace ugx {

constexpr double kPi = 3.14159265358979323846;
constexpr int N_DOF = 3;  // translational + internal degrees of freedom (monatomic)

// ------------------------------------------------------------------------
// storage types of f: FP64, FP32 or bfloat16 (all arithmetic is FP64)
// ------------------------------------------------------------------------
struct bf16s {
    unsigned short bits;
};
__device__ __forceinline__ double to_f64(double x) { return x; }
__device__ __forceinline__ double to_f64(float x) { return (double)x; }
__device__ __forceinline__ double to_f64(bf16s x) { return (double)__uint_as_float((unsigned)x.bits << 16); }

// The value itself, opaque to the compiler: a multiply that produced it can
// no longer be fused into a later add or subtract, so arithmetic on it sees
// the rounded value -- as it does when the value is read back from memory.
__device__ __forceinline__ double opaque(double x)
{
    asm volatile("" : "+v"(x));
    return x;
}

template <typename FT> __device__ __forceinline__ FT from_f64(double x);
template <> __device__ __forceinline__ double from_f64<double>(double x) { return x; }
template <> __device__ __forceinline__ float from_f64<float>(double x) { return (float)x; }
// Round to nearest, ties to even, directly from FP64 to the 8 significant
// bits of bfloat16: round the FP64 significand at its bit 45, then the
// result is exact in FP32 and its upper half is the bfloat16 pattern
// (values below the FP32 normal range are flushed to signed zero).
template <> __device__ __forceinline__ bf16s from_f64<bf16s>(double x)
{
    if (x != x) return bf16s{0x7fc0};
    unsigned long long u = (unsigned long long)__double_as_longlong(x);
    u += 0x00000fffffffffffull + ((u >> 45) & 1ull);
    u &= ~0x00001fffffffffffull;
    const double r = __longlong_as_double((long long)u);
    const float f = fabs(r) < 1.1754943508222875e-38 ? copysignf(0.0f, (float)r) : (float)r;
    return bf16s{(unsigned short)(__float_as_uint(f) >> 16)};
}

// ------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------
template <int D> __device__ __forceinline__ double pow_lam_pi(double lam)
{
    double r = lam / kPi;
    if constexpr (D == 2) return r;
    else return r * sqrt(r);
}

template <int BS, int N, typename Op>
__device__ __forceinline__ void block_reduce(double (&v)[N], double *lds, Op op)
{
    // butterfly inside the wavefront, then the wavefront results in fixed order
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[n] = op(v[n], __shfl_xor(v[n], off, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int n = 0; n < N; ++n) lds[wid * N + n] = v[n];
    __syncthreads();
#pragma unroll
    for (int n = 0; n < N; ++n) {
        double s = lds[n];
#pragma unroll
        for (int w = 1; w < BS / 64; ++w) s = op(s, lds[w * N + n]);
        v[n] = s;
    }
    __syncthreads();
}

// The same reduction for wide workgroups (many wavefronts): one thread per
// value sums the wavefronts' results, in the same fixed order, and the
// totals are broadcast through LDS; lds holds (BS / 64 + 1) * N doubles.
template <int BS, int N, typename Op>
__device__ __forceinline__ void block_reduce_wide(double (&v)[N], double *lds, Op op)
{
    constexpr int NWAVE = BS / 64;
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[n] = op(v[n], __shfl_xor(v[n], off, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int n = 0; n < N; ++n) lds[wid * N + n] = v[n];
    __syncthreads();
    if ((int)threadIdx.x < N) {
        double s = lds[threadIdx.x];
        for (int w = 1; w < NWAVE; ++w) s = op(s, lds[w * N + threadIdx.x]);
        lds[NWAVE * N + threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] = lds[NWAVE * N + n];
    __syncthreads();
}

struct OpAdd {
    __device__ double operator()(double a, double b) const { return a + b; }
};
struct OpMax {
    __device__ double operator()(double a, double b) const { return fmax(a, b); }
};

template <int D> struct Prim {
    double rho, U[D], lam;
};

template <int D> __device__ __forceinline__ Prim<D> to_prim(const double *W)
{
    Prim<D> p;
    p.rho = W[0];
    double ke = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        p.U[d] = W[1 + d] / p.rho;
        ke += p.U[d] * p.U[d];
    }
    p.lam = N_DOF * p.rho / (4.0 * (W[D + 1] - 0.5 * p.rho * ke));
    return p;
}

__device__ __forceinline__ double collision_time(double rho, double lam, double mu_ref, double omega)
{
    double T = 1.0 / lam;
    return mu_ref * pow(T, omega) / (0.5 * rho * T);
}

// Reduced Maxwellian and Shakhov correction at u (Section 2.2):
// H = pref e^{-lam c^2}, B = M/(2 lam) H,
// H+ = shk (c.q)(2 lam c^2 - 2 - D) H, B+ = shk (c.q)(2 lam c^2 - D) M H / (2 lam)
template <int D>
__device__ __forceinline__ void equilibrium(const double (&u)[D], const double (&U)[D], double lam, double pref,
                                            double shk, const double (&q)[D], double &Hp, double &Bp)
{
    constexpr int M = Dim<D>::M;
    double c2 = 0.0, cq = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double c = u[d] - U[d];
        c2 += c * c;
        cq += c * q[d];
    }
    double H = pref * exp(-lam * c2);
    double s = shk * cq;
    Hp = H + s * (2.0 * lam * c2 - 2.0 - D) * H;
    if constexpr (M > 0) {
        double B = (M / (2.0 * lam)) * H;
        Bp = B + s * (2.0 * lam * c2 - D) * B;
    } else {
        Bp = 0.0;
    }
}

// ------------------------------------------------------------------------
// limited least-squares slope of f_k in cell c (Section 3.1, step 2)
// ------------------------------------------------------------------------
// Reciprocal to full double precision: hardware estimate and two Newton steps.
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// The stencil of cell c at velocity k: its own value, then one value per face
// slot.  A slot without a neighbour (boundary face, or no face: nb = -1) reads
// the cell's own value, whose difference from it is exactly zero and whose
// least-squares weight is zero, so every load is issued and none sits behind a
// branch.  Loads take a uniform base and a 32-bit byte offset (a cell's slab
// is far below 4 GiB).  The sweep loads the next velocity's stencil while it
// works on the current one; limited_slope = load_stencil + slope_from.
template <typename FT>
__device__ __forceinline__ double load_at(const FT *__restrict__ base, unsigned idx)
{
    return to_f64(*reinterpret_cast<const FT *>(reinterpret_cast<const char *>(base) + idx * (unsigned)sizeof(FT)));
}

template <int D, typename FT>
__device__ __forceinline__ void load_stencil(const CellGeo<D> &g, int c, const FT *__restrict__ f, int nv, int k,
                                             double (&v0)[Dim<D>::NC], double (&vn)[Dim<D>::MF][Dim<D>::NC])
{
    constexpr int NC = Dim<D>::NC, MF = Dim<D>::MF;
    const FT *fcell = f + (size_t)c * NC * nv;
#pragma unroll
    for (int m = 0; m < NC; ++m) v0[m] = load_at(fcell, (unsigned)(m * nv + k));
#pragma unroll
    for (int j = 0; j < MF; ++j) {
        const int n = g.nb[j];
        const FT *fnb = f + (size_t)(n < 0 ? c : n) * NC * nv;
#pragma unroll
        for (int m = 0; m < NC; ++m) vn[j][m] = load_at(fnb, (unsigned)(m * nv + k));
    }
}

template <int D>
__device__ __forceinline__ void slope_from(const CellGeo<D> &g, int limiter, const double (&v0)[Dim<D>::NC],
                                           const double (&vn)[Dim<D>::MF][Dim<D>::NC], double (&fc)[Dim<D>::NC],
                                           double (&gr)[Dim<D>::NC][D])
{
    constexpr int NC = Dim<D>::NC, MF = Dim<D>::MF;
    // extremes of the differences f_j - f_i (0 for the cell itself): equal to
    // max_j f_j - f_i and min_j f_j - f_i, as rounding is monotone
    double up[NC], dn[NC];
#pragma unroll
    for (int m = 0; m < NC; ++m) {
        fc[m] = v0[m];
        up[m] = dn[m] = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) gr[m][d] = 0.0;
    }
    const int nf = g.nf;
    // a cell has at least D + 1 faces; the slots beyond are skipped
#pragma unroll
    for (int j = 0; j < MF; ++j) {
        if (j > D && j >= nf) break;
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            const double df = vn[j][m] - fc[m];
#pragma unroll
            for (int d = 0; d < D; ++d) gr[m][d] = fma(g.lsq[j][d], df, gr[m][d]);
            up[m] = fmax(up[m], df);
            dn[m] = fmin(dn[m], df);
        }
    }
    if (!limiter) return;
    // phi = min(1, min over faces of the Venkatakrishnan factor), the
    // fractions compared by cross-multiplication (denominators are positive);
    // a face with no increment gives num = den and never wins
#pragma unroll
    for (int m = 0; m < NC; ++m) {
        double bn = 1.0, bd = 1.0;
#pragma unroll
        for (int j = 0; j < MF; ++j) {
            if (j >= nf) break;
            double dm = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) dm = fma(gr[m][d], g.dvec[j][d], dm);
            const double dp = dm > 0.0 ? up[m] : dn[m];
            const double dp2e = fma(dp, dp, g.eps2);
            const double num = fma(2.0 * dm, dp, dp2e);
            const double den = fma(dm, fma(2.0, dm, dp), dp2e);
            const bool take = num * bd < bn * den;
            bn = take ? num : bn;
            bd = take ? den : bd;
        }
        const double phi = bn * rcp_nr(bd);
#pragma unroll
        for (int d = 0; d < D; ++d) gr[m][d] *= phi;
    }
}

template <int D, typename FT>
__device__ __forceinline__ void limited_slope(const CellGeo<D> &g, int c, const FT *__restrict__ f, int nv, int k,
                                              int limiter, double (&fc)[Dim<D>::NC], double (&gr)[Dim<D>::NC][D])
{
    double v0[Dim<D>::NC], vn[Dim<D>::MF][Dim<D>::NC];
    load_stencil<D, FT>(g, c, f, nv, k, v0, vn);
    slope_from<D>(g, limiter, v0, vn, fc, gr);
}

// Shakhov equilibrium f+ = H + H+ (and B + B+) at u, given the reduced
// Maxwellian value H there (Section 2.2):
// H+ = shk (c.q)(2 lam c^2 - 2 - D) H, B = M/(2 lam) H,
// B+ = shk (c.q)(2 lam c^2 - D) B, with shk = 4 (1 - Pr) lam^2 / (5 rho).
template <int D>
__device__ __forceinline__ void shakhov(const double (&u)[D], const double (&U)[D], double lam, double shk,
                                        const double (&q)[D], double bh, double H, double &fh, double &fb)
{
    constexpr int M = Dim<D>::M;
    double c2 = 0.0, cq = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double c = u[d] - U[d];
        c2 = fma(c, c, c2);
        cq = fma(c, q[d], cq);
    }
    const double s = shk * cq, l2 = 2.0 * lam * c2;
    fh = fma(s * (l2 - 2.0 - D), H, H);
    if constexpr (M > 0) {
        const double B = bh * H;  // bh = M / (2 lam)
        fb = fma(s * (l2 - D), B, B);
    } else {
        fb = 0.0;
    }
}

// Time-integrated interface value of h (and b) at velocity u (Eq. fullSolution
// integrated over [0, dt]); val is the upwind reconstruction at the face,
// ug = u . grad of the upwind cell, H0 the reduced Maxwellian g0 at u.
template <int D>
__device__ __forceinline__ void interface_integral(const FaceEq<D> &e, const double (&u)[D], double u2, double H0,
                                                   const double (&val)[Dim<D>::NC], const double (&ug)[Dim<D>::NC],
                                                   double (&I)[Dim<D>::NC])
{
    constexpr int M = Dim<D>::M, NW = D + 2;
    double eqH, eqB;
    shakhov<D>(u, e.U, e.lam, e.shk, e.q, e.bh, H0, eqH, eqB);
    double Pd = 0.0, Ed = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double pa = e.a[d][0] + 0.5 * e.a[d][NW - 1] * u2;
#pragma unroll
        for (int c = 0; c < D; ++c) pa += e.a[d][1 + c] * u[c];
        Pd += u[d] * pa;
        Ed += u[d] * e.a[d][NW - 1];
    }
    double PA = e.A[0] + 0.5 * e.A[NW - 1] * u2;
#pragma unroll
    for (int c = 0; c < D; ++c) PA += e.A[1 + c] * u[c];
    if constexpr (M > 0) {
        const double B0 = e.bh * H0;
        const double xi4 = e.x4 * H0;  // int xi^4 g0 dxi
        const double gH = Pd * H0 + 0.5 * Ed * B0, gB = Pd * B0 + 0.5 * Ed * xi4;
        const double tH = PA * H0 + 0.5 * e.A[NW - 1] * B0, tB = PA * B0 + 0.5 * e.A[NW - 1] * xi4;
        I[0] = e.c[0] * val[0] + e.c[1] * ug[0] + e.c[2] * eqH + e.c[3] * gH + e.c[4] * tH;
        I[1] = e.c[0] * val[1] + e.c[1] * ug[1] + e.c[2] * eqB + e.c[3] * gB + e.c[4] * tB;
    } else {
        const double gH = Pd * H0, tH = PA * H0;
        I[0] = e.c[0] * val[0] + e.c[1] * ug[0] + e.c[2] * eqH + e.c[3] * gH + e.c[4] * tH;
    }
}

// ------------------------------------------------------------------------
// time step: per cell, the largest upwind outflow over the velocities
// ------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_cfl(Params p, double *cell_dt)
{
    const int i = blockIdx.x;
    const CellGeo<D> &g = static_cast<const CellGeo<D> *>(p.cgeo)[i];
    const FaceGeo<D> *fg = static_cast<const FaceGeo<D> *>(p.fgeo);
    double mx[1] = {0.0};
    for (int k = threadIdx.x; k < p.nv; k += 256) {
        double out = 0.0;
        for (int j = 0; j < g.nf; ++j) {
            const FaceGeo<D> &F = fg[g.face[j]];
            double un = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) un += p.u[d * p.nv + k] * F.n[d];
            if (g.side[j]) un = -un;
            if (un > 0.0) out += F.area * un;
        }
        mx[0] = fmax(mx[0], out);
    }
    __shared__ double lds[4];
    block_reduce<256>(mx, lds, OpMax{});
    if (threadIdx.x == 0) cell_dt[i] = mx[0] > 0.0 ? (1.0 / g.inv_vol) / mx[0] : DBL_MAX;
}

// ------------------------------------------------------------------------
// initial state: discrete Maxwellian of (rho, U, T)
// ------------------------------------------------------------------------
// One workgroup per cell, threads over its velocities (a thread per
// (cell, velocity) would exceed the 2^32 work-items of one grid dimension on
// the largest meshes).
template <int D, typename FT>
__global__ __launch_bounds__(256) void k_init(Params p, const double *__restrict__ prim0, FT *__restrict__ f)
{
    constexpr int NC = Dim<D>::NC;
    const int i = blockIdx.x;
    const double *pr = prim0 + (size_t)i * (D + 2);
    double U[D], zq[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        U[d] = pr[1 + d];
        zq[d] = 0.0;
    }
    const double lam = 1.0 / pr[D + 1];
    const double pref = pr[0] * pow_lam_pi<D>(lam);
    for (int k = threadIdx.x; k < p.nv; k += 256) {
        double u[D];
#pragma unroll
        for (int d = 0; d < D; ++d) u[d] = p.u[d * p.nv + k];
        double H, B;
        equilibrium<D>(u, U, lam, pref, 0.0, zq, H, B);
        f[((size_t)i * NC + 0) * p.nv + k] = from_f64<FT>(H);
        if constexpr (NC > 1) f[((size_t)i * NC + 1) * p.nv + k] = from_f64<FT>(B);
    }
}

// ------------------------------------------------------------------------
// W and q as direct discrete moments of f (start, or after a set_f)
// ------------------------------------------------------------------------
template <int D, typename FT>
__global__ __launch_bounds__(256) void k_moments(Params p, const FT *__restrict__ f)
{
    constexpr int NC = Dim<D>::NC, NW = D + 2;
    const int i = blockIdx.x;
    __shared__ double lds[4 * NW];
    double m[NW];
#pragma unroll
    for (int n = 0; n < NW; ++n) m[n] = 0.0;
    for (int k = threadIdx.x; k < p.nv; k += 256) {
        double h = to_f64(f[((size_t)i * NC) * p.nv + k]);
        double b = NC > 1 ? to_f64(f[((size_t)i * NC + NC - 1) * p.nv + k]) : 0.0;
        double w = p.w[k], u2 = 0.0;
        m[0] += w * h;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            double ud = p.u[d * p.nv + k];
            m[1 + d] += w * ud * h;
            u2 += ud * ud;
        }
        m[NW - 1] += w * 0.5 * (u2 * h + b);
    }
    block_reduce<256>(m, lds, OpAdd{});
    Prim<D> pr = to_prim<D>(m);
    double qq[D];
#pragma unroll
    for (int d = 0; d < D; ++d) qq[d] = 0.0;
    for (int k = threadIdx.x; k < p.nv; k += 256) {
        double h = to_f64(f[((size_t)i * NC) * p.nv + k]);
        double b = NC > 1 ? to_f64(f[((size_t)i * NC + NC - 1) * p.nv + k]) : 0.0;
        double c[D], c2 = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            c[d] = p.u[d * p.nv + k] - pr.U[d];
            c2 += c[d] * c[d];
        }
        double wt = 0.5 * p.w[k] * (c2 * h + b);
#pragma unroll
        for (int d = 0; d < D; ++d) qq[d] += wt * c[d];
    }
    block_reduce<256>(qq, lds, OpAdd{});
    if (threadIdx.x == 0) {
#pragma unroll
        for (int n = 0; n < NW; ++n) p.W[(size_t)i * NW + n] = m[n];
#pragma unroll
        for (int d = 0; d < D; ++d) p.q[(size_t)i * D + d] = qq[d];
    }
}

// ------------------------------------------------------------------------
// Algorithm 1, macroscopic reconstruction: limited gradients of the conservative variables
// ------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void cell_grad(const Params p, int i)
{
    constexpr int NW = D + 2, MF = Dim<D>::MF;
    if (i >= p.nc) return;
    const CellGeo<D> &g = static_cast<const CellGeo<D> *>(p.cgeo)[i];
    const int nf = g.nf;
    // the cell's W and its neighbours' (the cell's own where a slot has no
    // neighbour: its difference is exactly zero), all loads issued at once
    double Wi[NW], Wn[MF][NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) Wi[m] = p.W[(size_t)i * NW + m];
#pragma unroll
    for (int j = 0; j < MF; ++j) {
        const int n = j < nf ? g.nb[j] : -1;
        const size_t src = (size_t)(n < 0 ? i : n) * NW;
#pragma unroll
        for (int m = 0; m < NW; ++m) Wn[j][m] = p.W[src + m];
    }
    double gr[NW][D];
#pragma unroll
    for (int m = 0; m < NW; ++m) {
        double mx = Wi[m], mn = Wi[m];
#pragma unroll
        for (int d = 0; d < D; ++d) gr[m][d] = 0.0;
#pragma unroll
        for (int j = 0; j < MF; ++j) {
            if (j >= nf) break;
            const double wj = Wn[j][m];
#pragma unroll
            for (int d = 0; d < D; ++d) gr[m][d] += g.lsq[j][d] * (wj - Wi[m]);
            mx = fmax(mx, wj);
            mn = fmin(mn, wj);
        }
        if (p.limiter) {
            double phi = 1.0;
#pragma unroll
            for (int j = 0; j < MF; ++j) {
                if (j >= nf) break;
                double dm = 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) dm += gr[m][d] * g.dvec[j][d];
                if (dm == 0.0) continue;
                double dp = dm > 0.0 ? mx - Wi[m] : mn - Wi[m];
                double ph = (dp * dp + g.eps2 + 2.0 * dm * dp) / (dp * dp + 2.0 * dm * dm + dm * dp + g.eps2);
                phi = fmin(phi, ph);
            }
#pragma unroll
            for (int d = 0; d < D; ++d) gr[m][d] *= phi;
        }
    }
    // first order where a reconstructed face state is not physical
    bool bad = false;
#pragma unroll
    for (int j = 0; j < MF; ++j) {
        if (j >= nf) break;
        double Wf[NW], ke = 0.0;
#pragma unroll
        for (int m = 0; m < NW; ++m) {
            Wf[m] = Wi[m];
#pragma unroll
            for (int d = 0; d < D; ++d) Wf[m] += gr[m][d] * g.dvec[j][d];
        }
#pragma unroll
        for (int d = 0; d < D; ++d) ke += Wf[1 + d] * Wf[1 + d];
        if (!(Wf[0] > 0.0) || !(Wf[NW - 1] - 0.5 * ke / Wf[0] > 0.0)) bad = true;
    }
#pragma unroll
    for (int m = 0; m < NW; ++m)
#pragma unroll
        for (int d = 0; d < D; ++d) p.gW[((size_t)i * NW + m) * D + d] = bad ? 0.0 : gr[m][d];
}

template <int D>
__global__ __launch_bounds__(256) void k_cell_grad(Params p)
{
    cell_grad<D>(p, blockIdx.x * 256 + threadIdx.x);
}

// ------------------------------------------------------------------------
// Algorithm 1, interface equilibrium state and time coefficients
// ------------------------------------------------------------------------
// Solve <psi (a . psi)>_{g} = Delta for a Maxwellian (rho-normalised
// moments, N = 3 degrees of freedom), in closed form.
template <int D>
__device__ void slope_solve(const double (&U)[D], double lam, const double *Dl, double *a)
{
    constexpr int NW = D + 2;
    double U2 = 0.0, UR = 0.0, R[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        U2 += U[d] * U[d];
        R[d] = Dl[1 + d] - U[d] * Dl[0];
        UR += U[d] * R[d];
    }
    const double K2 = U2 + N_DOF / (2.0 * lam);
    const double RE = 2.0 * Dl[NW - 1] - K2 * Dl[0];
    const double aE = (4.0 * lam * lam / N_DOF) * (RE - 2.0 * UR);
    double Ua = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        a[1 + d] = 2.0 * lam * R[d] - U[d] * aE;
        Ua += U[d] * a[1 + d];
    }
    a[NW - 1] = aE;
    a[0] = Dl[0] - Ua - 0.5 * aE * K2;
}

// -sum_d <psi u_d (a^d . psi)>_g  (Gaussian moments to fifth order)
template <int D>
__device__ void compat_rhs(const double (&U)[D], double lam, const double (*a)[D + 2], double *r)
{
    constexpr int NW = D + 2, N = N_DOF;
    const double s = 1.0 / (2.0 * lam);
    double U2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) U2 += U[d] * U[d];
    const double E = 0.5 * (U2 + N * s);
    const double c4 = U2 + (N + 4) * s, c2 = s * (U2 + (N + 2) * s);
    const double e2 = 0.25 * (U2 * U2 + 2.0 * (N + 4) * s * U2 + (N + 2) * (N + 4) * s * s);
    for (int m = 0; m < NW; ++m) r[m] = 0.0;
    for (int d = 0; d < D; ++d) {
        const double *ad = a[d];
        const double a0 = ad[0], aE = ad[NW - 1];
        // row 0
        double t = U[d] * a0 + U[d] * (E + s) * aE;
        for (int c = 0; c < D; ++c) t += (U[c] * U[d] + (c == d ? s : 0.0)) * ad[1 + c];
        r[0] -= t;
        // momentum rows
        for (int b = 0; b < D; ++b) {
            double tb = (U[b] * U[d] + (b == d ? s : 0.0)) * a0;
            for (int c = 0; c < D; ++c) {
                double m3 = U[b] * U[c] * U[d] +
                            s * ((c == d ? U[b] : 0.0) + (b == d ? U[c] : 0.0) + (b == c ? U[d] : 0.0));
                tb += m3 * ad[1 + c];
            }
            tb += 0.5 * (U[b] * U[d] * c4 + (b == d ? c2 : 0.0)) * aE;
            r[1 + b] -= tb;
        }
        // energy row
        double te = U[d] * (E + s) * a0 + U[d] * e2 * aE;
        for (int c = 0; c < D; ++c) te += 0.5 * (U[c] * U[d] * c4 + (c == d ? c2 : 0.0)) * ad[1 + c];
        r[NW - 1] -= te;
    }
}

__device__ void time_integrals(double dt, double tau, double *c)
{
    const double x = dt / tau;
    if (x < 1.0) {
        // Taylor series (the closed forms cancel catastrophically for small x)
        double term[31];
        term[0] = 1.0;
        for (int m = 1; m <= 30; ++m) term[m] = term[m - 1] * x / m;
        double s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0;
        for (int m = 30; m >= 1; --m) {
            const double t = (m & 1) ? term[m] : -term[m];
            s1 += t;
            if (m >= 2) {
                s2 += (m - 1) * t;
                s3 -= t;
            }
            if (m >= 3) {
                s4 -= (m - 2) * t;
                s5 += t;
            }
        }
        c[0] = tau * s1;
        c[1] = tau * tau * s2;
        c[2] = tau * s3;
        c[3] = tau * tau * s4;
        c[4] = tau * tau * s5;
    } else {
        const double e = exp(-x), ome = -expm1(-x);
        c[0] = tau * ome;
        c[1] = tau * dt * e - tau * tau * ome;
        c[2] = dt - tau * ome;
        c[3] = 2.0 * tau * tau * ome - tau * dt * (1.0 + e);
        c[4] = 0.5 * dt * dt - tau * dt + tau * tau * ome;
    }
}

template <int D>
__device__ __forceinline__ void face_eq(const Params p, int f)
{
    constexpr int NW = D + 2;
    if (f >= p.nf) return;
    const FaceGeo<D> &F = static_cast<const FaceGeo<D> *>(p.fgeo)[f];
    FaceEq<D> &e = static_cast<FaceEq<D> *>(p.feq)[f];
    e.dt = p.dt;
    e.hdt2 = 0.5 * p.dt * p.dt;
    if (F.bc != 0) {
        // boundary: store the Maxwellian the incoming particles come from
        double rho, U[D], lam;
        if (F.bc == 2) {
            Prim<D> pr = to_prim<D>(p.W + (size_t)F.l * NW);
            rho = pr.rho;
            lam = pr.lam;
            for (int d = 0; d < D; ++d) U[d] = pr.U[d];
        } else {
            const double *bp = p.bc_prim + (size_t)F.bcid * NW;
            rho = F.bc == 3 ? 1.0 : bp[0];
            for (int d = 0; d < D; ++d) U[d] = bp[1 + d];
            lam = 1.0 / bp[NW - 1];
        }
        e.rho = rho;
        e.lam = lam;
        for (int d = 0; d < D; ++d) e.U[d] = U[d];
        e.pref = rho * pow_lam_pi<D>(lam);
        e.shk = 0.0;
        e.bh = Dim<D>::M / (2.0 * lam);
        e.x4 = 0.0;
        return;
    }
    // reconstructed states on both sides
    double Wl[NW], Wr[NW];
    for (int m = 0; m < NW; ++m) {
        Wl[m] = p.W[(size_t)F.l * NW + m];
        Wr[m] = p.W[(size_t)F.r * NW + m];
        for (int d = 0; d < D; ++d) {
            Wl[m] += p.gW[((size_t)F.l * NW + m) * D + d] * F.dl[d];
            Wr[m] += p.gW[((size_t)F.r * NW + m) * D + d] * F.dr[d];
        }
    }
    // W0 from the two half-Maxwellians in the face-normal frame
    double W0[NW];
    for (int m = 0; m < NW; ++m) W0[m] = 0.0;
    for (int side = 0; side < 2; ++side) {
        Prim<D> pr = to_prim<D>(side == 0 ? Wl : Wr);
        double Un = 0.0;
        for (int d = 0; d < D; ++d) Un += pr.U[d] * F.n[d];
        double Ut[D], ut2 = 0.0;
        for (int d = 0; d < D; ++d) {
            Ut[d] = pr.U[d] - Un * F.n[d];
            ut2 += Ut[d] * Ut[d];
        }
        const double t = sqrt(pr.lam) * Un;
        const double g = exp(-pr.lam * Un * Un) / (2.0 * sqrt(kPi * pr.lam));
        double m0, m1;
        if (side == 0) {
            m0 = 0.5 * erfc(-t);
            m1 = Un * m0 + g;
        } else {
            m0 = 0.5 * erfc(t);
            m1 = Un * m0 - g;
        }
        const double m2 = Un * m1 + m0 / (2.0 * pr.lam);
        W0[0] += pr.rho * m0;
        for (int d = 0; d < D; ++d) W0[1 + d] += pr.rho * (m1 * F.n[d] + Ut[d] * m0);
        W0[NW - 1] += 0.5 * pr.rho * (m2 + (ut2 + (N_DOF - 1) / (2.0 * pr.lam)) * m0);
    }
    Prim<D> p0 = to_prim<D>(W0);
    e.rho = p0.rho;
    e.lam = p0.lam;
    for (int d = 0; d < D; ++d) e.U[d] = p0.U[d];
    e.pref = p0.rho * pow_lam_pi<D>(p0.lam);
    e.shk = 4.0 * (1.0 - p.Pr) * p0.lam * p0.lam / (5.0 * p0.rho);
    e.bh = Dim<D>::M / (2.0 * p0.lam);
    e.x4 = Dim<D>::M * (Dim<D>::M + 2) / (4.0 * p0.lam * p0.lam);
    // spatial slopes from the averaged limited gradients
    for (int d = 0; d < D; ++d) {
        double Dl[NW];
        for (int m = 0; m < NW; ++m)
            Dl[m] = 0.5 * (p.gW[((size_t)F.l * NW + m) * D + d] + p.gW[((size_t)F.r * NW + m) * D + d]) / p0.rho;
        slope_solve<D>(p0.U, p0.lam, Dl, e.a[d]);
    }
    double rhs[NW];
    compat_rhs<D>(p0.U, p0.lam, e.a, rhs);
    slope_solve<D>(p0.U, p0.lam, rhs, e.A);
    for (int d = 0; d < D; ++d) e.q[d] = 0.5 * (p.q[(size_t)F.l * D + d] + p.q[(size_t)F.r * D + d]);
    const double tau0 = collision_time(p0.rho, p0.lam, p.mu_ref, p.omega);
    time_integrals(p.dt, tau0, e.c);
}

template <int D>
__global__ __launch_bounds__(128) void k_face_eq(Params p)
{
    face_eq<D>(p, blockIdx.x * 128 + threadIdx.x);
}

// ------------------------------------------------------------------------
// Algorithm 1 from the velocity loop on, fused: the sweep over one cell's velocity slab
// ------------------------------------------------------------------------
// Unit-density Gaussian exp(-lam |u_k - U|^2).  On a Cartesian velocity grid
// it is the product of one-dimensional factors, tabulated in LDS once per
// workgroup (nx + ny [+ nz] exponentials instead of nx * ny [* nz]).
template <int D, bool TENSOR> struct Gauss {
    const double *tab;  // LDS tables, ntab doubles each
    int ntab;
    int off1, off2;     // start of the y and z axes inside a table
    __device__ __forceinline__ double operator()(int t, unsigned kx, const double (&u)[D], double lam,
                                                 const double *U) const
    {
        if constexpr (TENSOR) {
            const double *tb = tab + t * ntab;
            double g = tb[kx & 1023u] * tb[off1 + ((kx >> 10) & 1023u)];
            if constexpr (D == 3) g *= tb[off2 + (kx >> 20)];
            return g;
        } else {
            double c2 = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const double c = u[d] - U[d];
                c2 += c * c;
            }
            return exp(-lam * c2);
        }
    }
};

// One workgroup per cell; threads stride over the cell's velocities.
//   wall:   (wall cells only) incident and unit-density reflected mass fluxes
//           summed over velocities -> wall density;
//   pass 1: for each velocity, limited slopes (own cell, and the upwind
//           neighbour where it is upwind), the time-integrated flux through
//           every face, the stage-1 value -> written to f_out; moments of the
//           net outflow accumulated on the fly;
//   macro:  workgroup reduction -> W^{n+1}, tau^{n+1};
//   heat:   each thread re-reads its stage-1 values -> q^{n+1};
//   pass 2: each thread re-reads its stage-1 values, applies stage 2 and
//           writes f^{n+1}.
// Pass 1 parks the stage-1 values in LDS when the cell's slab fits there
// beside the tables with four workgroups per CU (then f_out is written once),
// otherwise in f_out itself.
#ifndef UGKS_XCDS
#define UGKS_XCDS 8  // accelerator complex dies of an MI355X
#endif
#ifndef UGKS_XCD_RUN
#define UGKS_XCD_RUN 32
#endif
// S1L: the stage-1 values of the cell are kept in LDS (when the slab fits
// beside the tables without costing occupancy), else in f_out until stage 2.
// Workgroups are dealt to the XCDs round-robin; hand each XCD runs of
// UGKS_XCD_RUN consecutive cells, so that mesh neighbours (whose slabs every
// workgroup re-reads) mostly meet in the same L2 while the runs, interleaved
// over the XCDs, keep the load balanced.  b is the workgroup's index within
// its case's grid, which starts at a multiple of UGKS_XCDS * UGKS_XCD_RUN.
__device__ __forceinline__ int xcd_cell(int b)
{
    const int t = b / UGKS_XCDS;
    return ((t / UGKS_XCD_RUN) * UGKS_XCDS + b % UGKS_XCDS) * UGKS_XCD_RUN + t % UGKS_XCD_RUN;
}

// Per-cell constants of a step (uniform in the workgroup): W^n, the
// primitive state, tau^n, q^n and the coefficients of f+^n and of the source.
template <int D> struct CellStep {
    static constexpr int NW = D + 2;
    double Wn[NW];
    Prim<D> pn;
    double qn[D];
    double pref_n, shk_n, hdt_tau, bh_n;
};

template <int D> __device__ __forceinline__ CellStep<D> cell_step(const Params &p, int i)
{
    constexpr int NW = D + 2;
    CellStep<D> s;
#pragma unroll
    for (int m = 0; m < NW; ++m) s.Wn[m] = p.W[(size_t)i * NW + m];
    s.pn = to_prim<D>(s.Wn);
    const double tau_n = collision_time(s.pn.rho, s.pn.lam, p.mu_ref, p.omega);
#pragma unroll
    for (int d = 0; d < D; ++d) s.qn[d] = p.q[(size_t)i * D + d];
    s.pref_n = s.pn.rho * pow_lam_pi<D>(s.pn.lam);
    s.shk_n = 4.0 * (1.0 - p.Pr) * s.pn.lam * s.pn.lam / (5.0 * s.pn.rho);
    s.hdt_tau = 0.5 * p.dt / tau_n;
    s.bh_n = Dim<D>::M / (2.0 * s.pn.lam);
    return s;
}

// One-dimensional Gaussian factors of every face's Maxwellian and of f+^n
// (tables 0..MF-1: the face slots, table MF: the cell); no barrier inside.
template <int D, int BS>
__device__ __forceinline__ void fill_tables(const Params &p, const CellGeo<D> &gi, double lam_c, double U0, double U1,
                                            double U2, double *tab)
{
    constexpr int NT = Dim<D>::MF + 1;
    const FaceEq<D> *fe = static_cast<const FaceEq<D> *>(p.feq);
    const int ntab = p.ntab, nf = gi.nf;
    for (int t = threadIdx.x; t < NT * ntab; t += BS) {
        const int which = t / ntab, idx = t - which * ntab;
        const int ax = idx < p.n1d[0] ? 0 : (idx < p.n1d[0] + p.n1d[1] ? 1 : 2);
        double lam, Ud;
        if (which < nf) {
            const FaceEq<D> &e = fe[gi.face[which]];
            lam = e.lam;
            Ud = e.U[0];
            if (ax == 1) Ud = e.U[1];
            if (D == 3 && ax == 2) Ud = e.U[D - 1];
        } else {
            lam = lam_c;
            Ud = ax == 0 ? U0 : (ax == 1 ? U1 : U2);
        }
        const double c = p.u1d[idx] - Ud;
        tab[t] = exp(-lam * c * c);
    }
}

// (the cell's state passed as scalars: a choice between fields of a
// structure would become a load at a chosen address, which keeps the
// structure in scratch memory)
template <int D, int BS>
__device__ __forceinline__ void fill_tables(const Params &p, const CellGeo<D> &gi, const Prim<D> &pn, double *tab)
{
    fill_tables<D, BS>(p, gi, pn.lam, pn.U[0], pn.U[1], pn.U[D - 1], tab);
}

template <int D> __device__ __forceinline__ int has_wall_face(const Params &p, const CellGeo<D> &gi)
{
    const FaceGeo<D> *fg = static_cast<const FaceGeo<D> *>(p.fgeo);
    int w = 0;
    for (int j = 0; j < gi.nf; ++j) w |= (fg[gi.face[j]].bc == 3);
    return w;
}

// Algorithm 1's boundary flux (wall density), for a cell with a wall face: the incident
// particles' mass flux and the unit-density reflected flux, summed over
// velocities; rho_w makes the net mass flux through the wall vanish
// (Eq. maxWalldes).  Knowing rho_w up front, the sweep adds the reflected
// particles directly.  Workgroup-wide (contains barriers).
template <int D, typename FT, int BS, bool TENSOR>
__device__ __forceinline__ void wall_density(const Params &p, const CellGeo<D> &gi, int i, const FT *__restrict__ fin,
                                             const Gauss<D, TENSOR> &gauss, double *red, double (&rho_w)[Dim<D>::MF])
{
    constexpr int NC = Dim<D>::NC, MF = Dim<D>::MF;
    const FaceGeo<D> *fg = static_cast<const FaceGeo<D> *>(p.fgeo);
    const FaceEq<D> *fe = static_cast<const FaceEq<D> *>(p.feq);
    const int nv = p.nv, nf = gi.nf;
    const double dt = p.dt;
    double wsum[2 * MF];
#pragma unroll
    for (int j = 0; j < 2 * MF; ++j) wsum[j] = 0.0;
    for (int k = threadIdx.x; k < nv; k += BS) {
        double u[D];
#pragma unroll
        for (int d = 0; d < D; ++d) u[d] = p.u[d * nv + k];
        const unsigned kx = TENSOR ? (unsigned)p.kidx[k] : 0u;
        const double wk = p.w[k];
        double fi[NC], gri[NC][D];
        limited_slope<D, FT>(gi, i, fin, nv, k, p.limiter, fi, gri);
#pragma unroll
        for (int j = 0; j < MF; ++j) {
            if (j >= nf) break;
            const FaceGeo<D> &F = fg[gi.face[j]];
            if (F.bc != 3) continue;
            double un = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) un += u[d] * F.n[d];
            if (un > 0.0) {
                double v = fi[0], ug = 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    v += gri[0][d] * gi.dvec[j][d];
                    ug += u[d] * gri[0][d];
                }
                wsum[2 * j] += wk * un * (dt * v - 0.5 * dt * dt * ug);
            } else {
                const FaceEq<D> &e = fe[gi.face[j]];
                wsum[2 * j + 1] += wk * un * dt * e.pref * gauss(j, kx, u, e.lam, e.U);
            }
        }
    }
    block_reduce<BS>(wsum, red, OpAdd{});
#pragma unroll
    for (int j = 0; j < MF; ++j) rho_w[j] = (j < nf && wsum[2 * j + 1] != 0.0) ? -wsum[2 * j] / wsum[2 * j + 1] : 0.0;
}

// After pass 1 of cell i: W^{n+1} (Eq. macroscopicUpdata) from the reduced
// moments, tau^{n+1}, q^{n+1} from the stage-1 values re-read, then stage 2
// (Eq. microS2) and the single store of f^{n+1}; tab holds the cell's tables
// (its own f+ table is refreshed for t^{n+1}).  Workgroup-wide.
template <int D, typename FT, int BS, bool TENSOR>
__device__ __forceinline__ void finish_cell(const Params &p, int i, const CellStep<D> &cs, double (&mom)[D + 2],
                                            const FT *s1, double *red, double *tab, const Gauss<D, TENSOR> &gauss,
                                            FT *__restrict__ fout)
{
    constexpr int NC = Dim<D>::NC, MF = Dim<D>::MF, NW = D + 2;
    const CellGeo<D> &gi = static_cast<const CellGeo<D> *>(p.cgeo)[i];
    const int tid = threadIdx.x, nv = p.nv;
    const double dt = p.dt, Pr = p.Pr;
    const size_t base = (size_t)i * NC * nv;

    // Algorithm 1's macroscopic update: Eq. macroscopicUpdata, then tau at t^{n+1}
    block_reduce<BS>(mom, red, OpAdd{});
    double W1[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) W1[m] = cs.Wn[m] - mom[m] * gi.inv_vol;
    const Prim<D> p1 = to_prim<D>(W1);
    const double tau1 = collision_time(p1.rho, p1.lam, p.mu_ref, p.omega);

    // heat flux of the stage-1 distribution about U^{n+1} (each thread
    // re-reads the values it wrote)
    double qt[D];
#pragma unroll
    for (int d = 0; d < D; ++d) qt[d] = 0.0;
    for (int k = tid; k < nv; k += BS) {
        double c[D], c2 = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            c[d] = p.u[d * nv + k] - p1.U[d];
            c2 += c[d] * c[d];
        }
        const double h = to_f64(s1[k]);
        const double b = NC > 1 ? to_f64(s1[(size_t)(NC - 1) * nv + k]) : 0.0;
        const double wt = 0.5 * p.w[k] * (c2 * h + b);
#pragma unroll
        for (int d = 0; d < D; ++d) qt[d] += wt * c[d];
    }
    block_reduce<BS>(qt, red, OpAdd{});
    double q1[D];
#pragma unroll
    for (int d = 0; d < D; ++d) q1[d] = qt[d] / (1.0 + Pr * dt / (2.0 * tau1));

    if constexpr (TENSOR) {
        // the cell's table now holds the factors of f+^{n+1}
        const int ntab = p.ntab;
        for (int idx = tid; idx < ntab; idx += BS) {
            const int ax = idx < p.n1d[0] ? 0 : (idx < p.n1d[0] + p.n1d[1] ? 1 : 2);
            double Ud = p1.U[0];
            if (ax == 1) Ud = p1.U[1];
            if (D == 3 && ax == 2) Ud = p1.U[D - 1];
            const double c = p.u1d[idx] - Ud;
            tab[MF * ntab + idx] = exp(-p1.lam * c * c);
        }
        __syncthreads();
    }

    // Algorithm 1's last step: Eq. microS2
    const double pref_1 = p1.rho * pow_lam_pi<D>(p1.lam);
    const double shk_1 = 4.0 * (1.0 - Pr) * p1.lam * p1.lam / (5.0 * p1.rho);
    const double a1 = 0.5 * dt / tau1, inv1 = 1.0 / (1.0 + a1);
    const double bh_1 = Dim<D>::M / (2.0 * p1.lam);
    for (int k = tid; k < nv; k += BS) {
        double u[D];
#pragma unroll
        for (int d = 0; d < D; ++d) u[d] = p.u[d * nv + k];
        const unsigned kx = TENSOR ? (unsigned)p.kidx[k] : 0u;
        double fp[2];
        const double H = pref_1 * gauss(MF, kx, u, p1.lam, p1.U);
        shakhov<D>(u, p1.U, p1.lam, shk_1, q1, bh_1, H, fp[0], fp[1]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            fout[base + (size_t)c * nv + k] = from_f64<FT>((to_f64(s1[(size_t)c * nv + k]) + a1 * fp[c]) * inv1);
        }
    }
    if (tid == 0) {
        bool ok = p1.rho > 0.0 && p1.lam > 0.0 && isfinite(p1.rho) && isfinite(p1.lam);
#pragma unroll
        for (int m = 0; m < NW; ++m) {
            ok = ok && isfinite(W1[m]);
            p.W[(size_t)i * NW + m] = W1[m];
            const double dw = W1[m] - cs.Wn[m];
            p.dW2[(size_t)i * NW + m] = dw * dw;
        }
#pragma unroll
        for (int d = 0; d < D; ++d) p.q[(size_t)i * D + d] = q1[d];
        if (!ok) {
            atomicOr(p.err, 1);
            atomicMin(p.err + 1, i);
        }
    }
}


// PF: the own cell's stencil of the next velocity is loaded one iteration
// ahead (20 more registers: used where they fit in the four-wave budget).
// CHUNK: the in-place mode's chunk kernel -- pass 1 over velocities
// [c0, c0 + cn) only, reading f^n and writing the stage-1 values to the ring
// (after writing the previous chunk's ring back into f), adding the chunk's
// moments to the cell's running sum (mom_part, started from zero by chunk 0),
// and the wall densities read from the wall kernel's array.
template <int D, typename FT, int BS, bool TENSOR, bool S1L, bool PF, bool CHUNK = false>
__device__ __forceinline__ void sweep_cell(const Params p, int i, const FT *__restrict__ fin, FT *__restrict__ fout,
                                           int c0 = 0, int cn = 0, int prev0 = 0, int prevn = 0, int ichunk = 0)
{
    constexpr int NC = Dim<D>::NC, MF = Dim<D>::MF, M = Dim<D>::M, NW = D + 2;
    constexpr int NT = MF + 1;  // Gaussian tables: one per face slot, one for the cell
    extern __shared__ double smem[];
    if (i >= p.nc) return;
    const int tid = threadIdx.x;
    const CellGeo<D> *cg = static_cast<const CellGeo<D> *>(p.cgeo);
    const FaceGeo<D> *fg = static_cast<const FaceGeo<D> *>(p.fgeo);
    const FaceEq<D> *fe = static_cast<const FaceEq<D> *>(p.feq);
    const CellGeo<D> &gi = cg[i];
    const int nv = p.nv, nf = gi.nf;
    const double dt = p.dt, Pr = p.Pr;
    const int ntab = TENSOR ? p.ntab : 0;
    double *red = smem + NT * ntab;
    const Gauss<D, TENSOR> gauss{smem, ntab, p.n1d[0], p.n1d[0] + p.n1d[1]};
    const size_t base = (size_t)i * NC * nv;
    constexpr int NRED = (NW > 2 * MF) ? NW : 2 * MF;
    // stage-1 values: LDS, f_out, or (chunk mode) the cell's ring, as
    // s1[c s1_stride + k - s1_off] for component c at velocity k
    FT *s1 = CHUNK ? static_cast<FT *>(p.ring) + (size_t)i * NC * p.chunk
                   : (S1L ? reinterpret_cast<FT *>(red + (BS / 64) * NRED) : fout + base);
    const size_t s1_stride = CHUNK ? (size_t)p.chunk : (size_t)nv;
    const int s1_off = CHUNK ? c0 : 0;
    const int k_end = CHUNK ? c0 + cn : nv;
    if constexpr (CHUNK) {
        // the previous chunk's stage-1 values go back into f (no workgroup
        // reads those velocities any more)
        for (int t = tid; t < prevn; t += BS)
#pragma unroll
            for (int c = 0; c < NC; ++c) fout[base + (size_t)c * nv + prev0 + t] = s1[(size_t)c * s1_stride + t];
    }

    // state at t^n
    double Wn[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) Wn[m] = p.W[(size_t)i * NW + m];
    const Prim<D> pn = to_prim<D>(Wn);
    const double tau_n = collision_time(pn.rho, pn.lam, p.mu_ref, p.omega);
    double qn[D];
#pragma unroll
    for (int d = 0; d < D; ++d) qn[d] = p.q[(size_t)i * D + d];
    const double pref_n = pn.rho * pow_lam_pi<D>(pn.lam);
    const double shk_n = 4.0 * (1.0 - Pr) * pn.lam * pn.lam / (5.0 * pn.rho);
    const double hdt_tau = 0.5 * dt / tau_n;
    const double bh_n = Dim<D>::M / (2.0 * pn.lam);

    int has_wall = 0;
    if constexpr (!CHUNK)
        for (int j = 0; j < nf; ++j) has_wall |= (fg[gi.face[j]].bc == 3);

    if constexpr (TENSOR) {
        // one-dimensional Gaussian factors of every face's Maxwellian and of f+^n
        for (int t = tid; t < NT * ntab; t += BS) {
            const int which = t / ntab, idx = t - which * ntab;
            const int ax = idx < p.n1d[0] ? 0 : (idx < p.n1d[0] + p.n1d[1] ? 1 : 2);
            double lam, Ud;
            if (which < nf) {
                const FaceEq<D> &e = fe[gi.face[which]];
                lam = e.lam;
                Ud = e.U[0];
                if (ax == 1) Ud = e.U[1];
                if (D == 3 && ax == 2) Ud = e.U[D - 1];
            } else {
                lam = pn.lam;
                Ud = pn.U[0];
                if (ax == 1) Ud = pn.U[1];
                if (D == 3 && ax == 2) Ud = pn.U[D - 1];
            }
            const double c = p.u1d[idx] - Ud;
            smem[t] = exp(-lam * c * c);
        }
    }
    __syncthreads();

    // Algorithm 1's boundary flux (wall density) first, for wall cells only: the incident
    // particles' mass flux and the unit-density reflected flux, summed over
    // velocities; rho_w makes the net mass flux through the wall vanish
    // (Eq. maxWalldes).  Knowing rho_w up front, the sweep below adds the
    // reflected particles directly.
    double rho_w[MF];
#pragma unroll
    for (int j = 0; j < MF; ++j) rho_w[j] = CHUNK ? p.rho_w[(size_t)i * MF + j] : 0.0;
    if (has_wall) {
        double wsum[2 * MF];
#pragma unroll
        for (int j = 0; j < 2 * MF; ++j) wsum[j] = 0.0;
        for (int k = tid; k < nv; k += BS) {
            double u[D];
#pragma unroll
            for (int d = 0; d < D; ++d) u[d] = p.u[d * nv + k];
            const unsigned kx = TENSOR ? (unsigned)p.kidx[k] : 0u;
            const double wk = p.w[k];
            double fi[NC], gri[NC][D];
            limited_slope<D, FT>(gi, i, fin, nv, k, p.limiter, fi, gri);
#pragma unroll
            for (int j = 0; j < MF; ++j) {
                if (j >= nf) break;
                const FaceGeo<D> &F = fg[gi.face[j]];
                if (F.bc != 3) continue;
                double un = 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) un += u[d] * F.n[d];
                if (un > 0.0) {
                    double v = fi[0], ug = 0.0;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        v += gri[0][d] * gi.dvec[j][d];
                        ug += u[d] * gri[0][d];
                    }
                    wsum[2 * j] += wk * un * (dt * v - 0.5 * dt * dt * ug);
                } else {
                    const FaceEq<D> &e = fe[gi.face[j]];
                    wsum[2 * j + 1] += wk * un * dt * e.pref * gauss(j, kx, u, e.lam, e.U);
                }
            }
        }
        block_reduce<BS>(wsum, red, OpAdd{});
#pragma unroll
        for (int j = 0; j < MF; ++j) rho_w[j] = (j < nf && wsum[2 * j + 1] != 0.0) ? -wsum[2 * j] / wsum[2 * j + 1] : 0.0;
    }

    // Algorithm 1's velocity loop: per velocity, limited slopes, interface fluxes,
    // stage 1; the moments of the net outflow give W^{n+1}
    double mom[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) mom[m] = 0.0;
    double pv0[NC], pvn[MF][NC];
    if (PF && s1_off + tid < k_end) load_stencil<D, FT>(gi, i, fin, nv, s1_off + tid, pv0, pvn);
    for (int k = s1_off + tid; k < k_end; k += BS) {
        double v0[NC], vn[MF][NC];
        if constexpr (PF) {
#pragma unroll
            for (int m = 0; m < NC; ++m) {
                v0[m] = pv0[m];
#pragma unroll
                for (int j = 0; j < MF; ++j) vn[j][m] = pvn[j][m];
            }
            if (k + BS < k_end) load_stencil<D, FT>(gi, i, fin, nv, k + BS, pv0, pvn);
        }
        double u[D], u2 = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            u[d] = p.u[d * nv + k];
            u2 += u[d] * u[d];
        }
        const unsigned kx = TENSOR ? (unsigned)p.kidx[k] : 0u;
        double fi[NC], gri[NC][D];
        if constexpr (PF) slope_from<D>(gi, p.limiter, v0, vn, fi, gri);
        else limited_slope<D, FT>(gi, i, fin, nv, k, p.limiter, fi, gri);
        double out[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c] = 0.0;
#pragma unroll
        for (int j = 0; j < MF; ++j) {
            if (j >= nf) break;
            const int f = gi.face[j];
            const FaceGeo<D> &F = fg[f];
            const FaceEq<D> &e = fe[f];
            double un = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) un += u[d] * F.n[d];
            double I[NC];
            if (F.bc == 0) {
                const bool self_up = (un > 0.0) == (gi.side[j] == 0);
                double val[NC], ug[NC];
                if (self_up) {
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        val[c] = fi[c];
                        ug[c] = 0.0;
#pragma unroll
                        for (int d = 0; d < D; ++d) {
                            val[c] += gri[c][d] * gi.dvec[j][d];
                            ug[c] += u[d] * gri[c][d];
                        }
                    }
                } else {
                    const int n = gi.nb[j];
                    const CellGeo<D> &gn = cg[n];
                    const int bj = gi.back[j];
                    double fn[NC], grn[NC][D];
                    limited_slope<D, FT>(gn, n, fin, nv, k, p.limiter, fn, grn);
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        val[c] = fn[c];
                        ug[c] = 0.0;
#pragma unroll
                        for (int d = 0; d < D; ++d) {
                            val[c] += grn[c][d] * gn.dvec[bj][d];
                            ug[c] += u[d] * grn[c][d];
                        }
                    }
                }
                const double H0 = e.pref * gauss(j, kx, u, e.lam, e.U);
                interface_integral<D>(e, u, u2, H0, val, ug, I);
            } else if (un > 0.0) {
                // outgoing through a wall or far-field face: free transport
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    double v = fi[c], ug = 0.0;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        v += gri[c][d] * gi.dvec[j][d];
                        ug += u[d] * gri[c][d];
                    }
                    I[c] = e.dt * v - e.hdt2 * ug;
                }
            } else {
                // incoming from the wall (density rho_w) or the ghost Maxwellian
                const double H = (F.bc == 3 ? rho_w[j] : 1.0) * e.pref * gauss(j, kx, u, e.lam, e.U);
                I[0] = e.dt * H;
                if constexpr (NC > 1) I[1] = e.dt * e.bh * H;
            }
            const double sa = (gi.side[j] ? -F.area : F.area) * un;
#pragma unroll
            for (int c = 0; c < NC; ++c) out[c] += sa * I[c];
        }
        // Eq. microS1 with the source at t^n
        double fpn[2];
        {
            const double H = pref_n * gauss(MF, kx, u, pn.lam, pn.U);
            shakhov<D>(u, pn.U, pn.lam, shk_n, qn, bh_n, H, fpn[0], fpn[1]);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
            s1[(size_t)c * s1_stride + (k - s1_off)] =
                from_f64<FT>(fi[c] - out[c] * gi.inv_vol + hdt_tau * (fpn[c] - fi[c]));
        // moments of the net outflow (Eq. macroscopicFlux summed over faces)
        const double wk = p.w[k];
        mom[0] += wk * out[0];
#pragma unroll
        for (int d = 0; d < D; ++d) mom[1 + d] += wk * u[d] * out[0];
        mom[NW - 1] += wk * 0.5 * (u2 * out[0] + (NC > 1 ? out[NC - 1] : 0.0));
    }

    // Algorithm 1's macroscopic update: Eq. macroscopicUpdata, then tau at t^{n+1}
    block_reduce<BS>(mom, red, OpAdd{});
    if constexpr (CHUNK) {
        // add this chunk's moments to the cell's sum; the chunks run one
        // launch after another, so the sum is taken in chunk order
        if (tid == 0) {
            double *acc = p.mom_part + (size_t)i * NW;
#pragma unroll
            for (int m = 0; m < NW; ++m) acc[m] = (ichunk == 0 ? 0.0 : acc[m]) + mom[m];
        }
        return;
    }
    double W1[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) W1[m] = Wn[m] - mom[m] * gi.inv_vol;
    const Prim<D> p1 = to_prim<D>(W1);
    const double tau1 = collision_time(p1.rho, p1.lam, p.mu_ref, p.omega);

    // heat flux of the stage-1 distribution about U^{n+1} (each thread
    // re-reads the values it wrote)
    double qt[D];
#pragma unroll
    for (int d = 0; d < D; ++d) qt[d] = 0.0;
    for (int k = tid; k < nv; k += BS) {
        double c[D], c2 = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            c[d] = p.u[d * nv + k] - p1.U[d];
            c2 += c[d] * c[d];
        }
        const double h = to_f64(s1[k]);
        const double b = NC > 1 ? to_f64(s1[(size_t)(NC - 1) * nv + k]) : 0.0;
        const double wt = 0.5 * p.w[k] * (c2 * h + b);
#pragma unroll
        for (int d = 0; d < D; ++d) qt[d] += wt * c[d];
    }
    block_reduce<BS>(qt, red, OpAdd{});
    double q1[D];
#pragma unroll
    for (int d = 0; d < D; ++d) q1[d] = qt[d] / (1.0 + Pr * dt / (2.0 * tau1));

    if constexpr (TENSOR) {
        // the cell's table now holds the factors of f+^{n+1}
        for (int idx = tid; idx < ntab; idx += BS) {
            const int ax = idx < p.n1d[0] ? 0 : (idx < p.n1d[0] + p.n1d[1] ? 1 : 2);
            double Ud = p1.U[0];
            if (ax == 1) Ud = p1.U[1];
            if (D == 3 && ax == 2) Ud = p1.U[D - 1];
            const double c = p.u1d[idx] - Ud;
            smem[MF * ntab + idx] = exp(-p1.lam * c * c);
        }
        __syncthreads();
    }

    // Algorithm 1's last step: Eq. microS2
    const double pref_1 = p1.rho * pow_lam_pi<D>(p1.lam);
    const double shk_1 = 4.0 * (1.0 - Pr) * p1.lam * p1.lam / (5.0 * p1.rho);
    const double a1 = 0.5 * dt / tau1, inv1 = 1.0 / (1.0 + a1);
    const double bh_1 = Dim<D>::M / (2.0 * p1.lam);
    for (int k = tid; k < nv; k += BS) {
        double u[D];
#pragma unroll
        for (int d = 0; d < D; ++d) u[d] = p.u[d * nv + k];
        const unsigned kx = TENSOR ? (unsigned)p.kidx[k] : 0u;
        double fp[2];
        const double H = pref_1 * gauss(MF, kx, u, p1.lam, p1.U);
        shakhov<D>(u, p1.U, p1.lam, shk_1, q1, bh_1, H, fp[0], fp[1]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            fout[base + (size_t)c * nv + k] = from_f64<FT>((to_f64(s1[(size_t)c * nv + k]) + a1 * fp[c]) * inv1);
        }
    }
    if (tid == 0) {
        bool ok = p1.rho > 0.0 && p1.lam > 0.0 && isfinite(p1.rho) && isfinite(p1.lam);
#pragma unroll
        for (int m = 0; m < NW; ++m) {
            ok = ok && isfinite(W1[m]);
            p.W[(size_t)i * NW + m] = W1[m];
            const double dw = W1[m] - Wn[m];
            p.dW2[(size_t)i * NW + m] = dw * dw;
        }
#pragma unroll
        for (int d = 0; d < D; ++d) p.q[(size_t)i * D + d] = q1[d];
        if (!ok) {
            atomicOr(p.err, 1);
            atomicMin(p.err + 1, i);
        }
    }
}

// ------------------------------------------------------------------------
// In-place mode (one f buffer): the velocities are swept in chunks.  A chunk
// kernel reads f^n of its velocities only (the cell's two-ring stencil),
// parks the stage-1 values in a ring buffer of one chunk per cell and adds
// the chunk's moments of the net outflow to the cell's running sum
// (mom_part: chunk 0 starts it from zero, the chunks run one launch after
// another); the next chunk kernel first writes its cell's ring back into f
// (no workgroup reads those velocities any more), and a final kernel writes
// the last chunk, reads that sum (W^{n+1}), forms q^{n+1} from the stage-1
// values now in f, and applies stage 2 in place.  This is the paper's in-place
// update of f (Section 3.2) with the ring as the only extra storage.  The
// wall density of every wall cell is reduced over all velocities first.
// ------------------------------------------------------------------------
template <int D, typename FT, int BS, bool TENSOR>
__global__ __launch_bounds__(BS) void k_wall_density(Params p, const FT *__restrict__ f)
{
    constexpr int MF = Dim<D>::MF, NT = MF + 1;
    extern __shared__ double smem[];
    const int i = xcd_cell(blockIdx.x);
    if (i >= p.nc) return;
    const CellGeo<D> &gi = static_cast<const CellGeo<D> *>(p.cgeo)[i];
    if (!has_wall_face<D>(p, gi)) return;  // uniform: the whole workgroup leaves
    const int ntab = TENSOR ? p.ntab : 0;
    const CellStep<D> cs = cell_step<D>(p, i);
    if constexpr (TENSOR) fill_tables<D, BS>(p, gi, cs.pn, smem);
    __syncthreads();
    const Gauss<D, TENSOR> gauss{smem, ntab, p.n1d[0], p.n1d[0] + p.n1d[1]};
    double rho_w[MF];
    wall_density<D, FT, BS, TENSOR>(p, gi, i, f, gauss, smem + NT * ntab, rho_w);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < MF; ++j) p.rho_w[(size_t)i * MF + j] = rho_w[j];
}

// The chunk sweep under the four-wave budget; the next velocity's stencil is
// prefetched for FP32 and BF16 f (with FP64 f the prefetch registers would
// spill: measured 8.9 against 7.7 ms per step on the cylinder).
template <int D, typename FT, int BS, bool TENSOR>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_sweep_chunk(
    Params p, FT *__restrict__ f, int c0, int cn, int prev0, int prevn, int ichunk)
{
    constexpr bool PF = TENSOR && sizeof(FT) < sizeof(double);
    sweep_cell<D, FT, BS, TENSOR, false, PF, true>(p, xcd_cell(blockIdx.x), f, f, c0, cn, prev0, prevn, ichunk);
}

template <int D, typename FT, int BS, bool TENSOR>
__global__ __launch_bounds__(BS) void k_sweep_finish(Params p, FT *__restrict__ f, int last0, int lastn)
{
    constexpr int NC = Dim<D>::NC, NW = D + 2;
    extern __shared__ double smem[];
    const int i = xcd_cell(blockIdx.x);
    if (i >= p.nc) return;
    const int tid = threadIdx.x, nv = p.nv, ch = p.chunk;
    const CellGeo<D> &gi = static_cast<const CellGeo<D> *>(p.cgeo)[i];
    const FT *ring = static_cast<const FT *>(p.ring) + (size_t)i * NC * ch;
    FT *fc = f + (size_t)i * NC * nv;
    for (int t = tid; t < lastn; t += BS)
#pragma unroll
        for (int c = 0; c < NC; ++c) fc[(size_t)c * nv + last0 + t] = ring[(size_t)c * ch + t];
    const int ntab = TENSOR ? p.ntab : 0;
    const CellStep<D> cs = cell_step<D>(p, i);
    if constexpr (TENSOR) fill_tables<D, BS>(p, gi, cs.pn, smem);
    // the chunks' moments, summed in chunk order by the chunk kernels
    double mom[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) mom[m] = p.mom_part[(size_t)i * NW + m];
    // block_reduce in finish_cell sums over the workgroup: only thread 0
    // carries the moments
    if (tid != 0)
#pragma unroll
        for (int m = 0; m < NW; ++m) mom[m] = 0.0;
    __syncthreads();
    constexpr int NT = Dim<D>::MF + 1;
    const Gauss<D, TENSOR> gauss{smem, ntab, p.n1d[0], p.n1d[0] + p.n1d[1]};
    finish_cell<D, FT, BS, TENSOR>(p, i, cs, mom, fc, smem + NT * ntab, smem, gauss, f);
}

template <int D, typename FT, int BS, bool TENSOR, bool S1L>
__global__ __launch_bounds__(BS) void k_sweep(Params p, const FT *__restrict__ fin, FT *__restrict__ fout)
{
    sweep_cell<D, FT, BS, TENSOR, S1L, false>(p, xcd_cell(blockIdx.x), fin, fout);
}

// Cartesian (tabulated) velocity sets: the same with the stencil prefetch,
// held to four waves per SIMD.
template <int D, typename FT, int BS, bool S1L>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_sweep_pf(Params p, const FT *__restrict__ fin, FT *__restrict__ fout)
{
    sweep_cell<D, FT, BS, true, S1L, true>(p, xcd_cell(blockIdx.x), fin, fout);
}

// ------------------------------------------------------------------------
// Push sweep (FP64 or FP32 f; two f buffers, or in place one f and a ring of
// one velocity chunk): each face flux once.
//
// Per velocity, the flux through an interior face needs the limited slope
// of the upwind cell only (Eq. fullSolution).  The cells are split into
// colours such that no two cells of a colour are neighbours or share a
// neighbour (distance-2 colouring), and one launch per colour advances its
// cells: a workgroup owns one cell's velocity slab (or a share of it, when
// a class is too small to fill the chip), rebuilds that cell's own limited
// slope, and for every face through which the cell is upwind
// at a velocity it evaluates the time-integrated flux once and adds it to
// the stage-1 accumulator of both cells (- F / |Omega_i| here, + F /
// |Omega_n| there) with hardware atomic adds that return nothing, so that
// the velocity loop never waits on an accumulator load.  Faces through which the cell is downwind are added by
// the neighbour in its own colour's launch.  No two workgroups of a launch
// touch the same accumulator, and the colours run in a fixed order, so the
// sums are deterministic; the accumulator holds, before the first colour,
// the stage-1 base f^n + (dt / 2 tau^n)(f+^n - f^n) of Eq. microS1 and,
// after the last, the stage-1 value itself.  A final kernel per cell then
// forms W^{n+1} = W^n + M(f~) - M(base) (M the moments (1, u, (|u|^2 h + b)
// / 2) summed over velocities: their difference is the sum over faces of
// the moments of the micro flux, Eqs. macroscopicFlux and
// macroscopicUpdata), tau^{n+1}, q^{n+1}, stage 2 (Eq. microS2) into the f
// buffer, and the next step's base (with its moments) into the
// accumulator.  Wall cells reduce the wall density over their velocities
// first (Eq. maxWalldes) and record the step's wall flux.
// ------------------------------------------------------------------------

// moments (1, u, (|u|^2 h + b) / 2) of one velocity's values, weighted
template <int D>
__device__ __forceinline__ void add_moments(double (&m)[D + 2], double w, const double (&u)[D], double u2, double h,
                                            double b)
{
    m[0] = fma(w, h, m[0]);
#pragma unroll
    for (int d = 0; d < D; ++d) m[1 + d] = fma(w * u[d], h, m[1 + d]);
    m[D + 1] = fma(0.5 * w, fma(u2, h, b), m[D + 1]);
}

// Two consecutive values of an f slab in one 2-wide access (the element
// offset even, so the access is aligned): the per-cell streaming kernels
// take velocities in pairs when the velocity count is even, which doubles
// the bytes each load keeps in flight.
template <typename FT> struct Vec2;
template <> struct Vec2<double> { using T = double2; };
template <> struct Vec2<float> { using T = float2; };
template <typename FT> __device__ __forceinline__ void load2(const FT *__restrict__ q, double &a, double &b)
{
    const typename Vec2<FT>::T v = *reinterpret_cast<const typename Vec2<FT>::T *>(q);
    a = to_f64(v.x);
    b = to_f64(v.y);
}
template <typename FT> __device__ __forceinline__ void store2(FT *__restrict__ q, FT a, FT b)
{
    typename Vec2<FT>::T v;
    v.x = a;
    v.y = b;
    *reinterpret_cast<typename Vec2<FT>::T *>(q) = v;
}
// bfloat16 pairs: one 32-bit word, the first value in its lower half
template <> __device__ __forceinline__ void load2<bf16s>(const bf16s *__restrict__ q, double &a, double &b)
{
    const unsigned v = *reinterpret_cast<const unsigned *>(q);
    a = to_f64(bf16s{(unsigned short)(v & 0xffffu)});
    b = to_f64(bf16s{(unsigned short)(v >> 16)});
}
template <> __device__ __forceinline__ void store2<bf16s>(bf16s *__restrict__ q, bf16s a, bf16s b)
{
    *reinterpret_cast<unsigned *>(q) = (unsigned)a.bits | ((unsigned)b.bits << 16);
}

// The push sweep's accumulator (the stage-1 sums) is kept in f's storage
// type, except with bfloat16 f: there it holds FP32, since a bfloat16 sum
// would round away most of every flux added to it.
template <typename FT> struct AccOf {
    using T = FT;
};
template <> struct AccOf<bf16s> {
    using T = float;
};

// velocity k's components of the velocity set
template <int D>
__device__ __forceinline__ void velocity(const Params &p, int k, double (&u)[D], double &u2)
{
    u2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        u[d] = p.u[d * p.nv + k];
        u2 = fma(u[d], u[d], u2);
    }
}

// Sum over the 64 lanes of a wavefront.  Every lane ends with the same
// bits: each butterfly step adds the same two values in both partner lanes.
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// The cell's own Gaussian factor table for (U, lam), filled by one
// wavefront into its own LDS region (ntab doubles), and a lookup in it.
template <int D>
__device__ __forceinline__ void fill_wave_table(const Params &p, const double (&U)[D], double lam, double *tb, int lane)
{
    const double U0 = U[0], U1 = U[1], U2 = U[D - 1];
    for (int idx = lane; idx < p.ntab; idx += 64) {
        const int ax = idx < p.n1d[0] ? 0 : (idx < p.n1d[0] + p.n1d[1] ? 1 : 2);
        const double Ud = ax == 0 ? U0 : (ax == 1 ? U1 : U2);
        const double c = p.u1d[idx] - Ud;
        tb[idx] = exp(-lam * c * c);
    }
    // the lanes' LDS writes before any lane of the wavefront reads them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <int D>
__device__ __forceinline__ double wave_table_gauss(const Params &p, const double *tb, unsigned kx)
{
    double g = tb[kx & 1023u] * tb[p.n1d[0] + ((kx >> 10) & 1023u)];
    if constexpr (D == 3) g *= tb[p.n1d[0] + p.n1d[1] + (kx >> 20)];
    return g;
}
template <int D, bool TENSOR>
__device__ __forceinline__ double own_gauss(const Params &p, const double *tb, unsigned kx, const double (&u)[D],
                                            double lam, const double (&U)[D])
{
    if constexpr (TENSOR) {
        return wave_table_gauss<D>(p, tb, kx);
    } else {
        double c2 = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double c = u[d] - U[d];
            c2 += c * c;
        }
        return exp(-lam * c2);
    }
}

// The per-cell streaming kernels of the push sweep run one wavefront per
// cell (four cells per workgroup, consecutive): the reductions over a
// cell's velocities are lane butterflies, with no workgroup barrier, so
// that each wavefront streams its slab without waiting for others.
constexpr int kPushCellsPerGroup = 4;

// Stage-1 base of cell i and its moments: acc = f + (dt / 2 tau)(f+ - f)
// from f^n, W^n, q^n (after a start, a restart or a step of another kind).
// V2: velocities in pairs (even velocity count).  Same lane order and
// arithmetic as the final kernel's second pass, so both give the same bits.
template <int D, typename FT, bool TENSOR, bool V2>
__global__ __launch_bounds__(256) void k_push_base(Params p, const FT *__restrict__ fin, typename AccOf<FT>::T *__restrict__ acc)
{
    using AT = typename AccOf<FT>::T;
    constexpr int NC = Dim<D>::NC, NW = D + 2, VW = V2 ? 2 : 1;
    extern __shared__ double smem[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = kPushCellsPerGroup * xcd_cell(blockIdx.x) + wv;
    if (i >= p.nc) return;
    const int nv = p.nv;
    const CellStep<D> cs = cell_step<D>(p, i);
    double *tb = smem + (size_t)wv * (TENSOR ? p.ntab : 0);
    if constexpr (TENSOR) fill_wave_table<D>(p, cs.pn.U, cs.pn.lam, tb, lane);
    const size_t base = (size_t)i * NC * nv;
    double mom[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) mom[m] = 0.0;
#pragma unroll 4
    for (int k0 = VW * lane; k0 < nv; k0 += VW * 64) {
        double f[VW][2];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if constexpr (V2)
                load2<FT>(fin + base + (size_t)c * nv + k0, f[0][c], f[1][c]);
            else
                f[0][c] = to_f64(fin[base + (size_t)c * nv + k0]);
        }
        AT sv[VW][2];
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const int k = k0 + e;
            double u[D], u2;
            velocity<D>(p, k, u, u2);
            const unsigned kx = TENSOR ? (unsigned)p.kidx[k] : 0u;
            double fp[2];
            const double H = cs.pref_n * own_gauss<D, TENSOR>(p, tb, kx, u, cs.pn.lam, cs.pn.U);
            shakhov<D>(u, cs.pn.U, cs.pn.lam, cs.shk_n, cs.qn, cs.bh_n, H, fp[0], fp[1]);
            double bv[2] = {0.0, 0.0};
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                sv[e][c] = from_f64<AT>(fma(cs.hdt_tau, fp[c] - f[e][c], f[e][c]));
                bv[c] = to_f64(sv[e][c]);
            }
            add_moments<D>(mom, p.w[k], u, u2, bv[0], NC > 1 ? bv[NC - 1] : 0.0);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if constexpr (V2)
                store2<AT>(acc + base + (size_t)c * nv + k0, sv[0][c], sv[1][c]);
            else
                acc[base + (size_t)c * nv + k0] = sv[0][c];
        }
    }
#pragma unroll
    for (int m = 0; m < NW; ++m) mom[m] = wave_sum(mom[m]);
    if (lane == 0)
#pragma unroll
        for (int m = 0; m < NW; ++m) p.mom_part[(size_t)i * NW + m] = mom[m];
}

// Wall faces of cell i (Section 2.5): per wall face, the incident particles'
// mass flux (free transport of the interior reconstruction) and the
// unit-density reflected one, summed over velocities, give rho_w
// (Eq. maxWalldes); the face's macroscopic flux over the step (incident +
// rho_w reflected) per unit area and time is recorded.  Workgroup-wide.
template <int D, typename FT, int BS, bool TENSOR>
__device__ __forceinline__ void push_wall(const Params &p, const CellGeo<D> &gi, int i, const FT *__restrict__ fin,
                                          const Gauss<D, TENSOR> &gauss, double *red, double (&rho_w)[Dim<D>::MF])
{
    constexpr int NC = Dim<D>::NC, MF = Dim<D>::MF, NW = D + 2;
    const FaceGeo<D> *fg = static_cast<const FaceGeo<D> *>(p.fgeo);
    const FaceEq<D> *fe = static_cast<const FaceEq<D> *>(p.feq);
    const int nv = p.nv, nf = gi.nf;
    const double dt = p.dt;
#pragma unroll
    for (int j = 0; j < MF; ++j) rho_w[j] = 0.0;
    for (int j = 0; j < nf; ++j) {
        const int f = gi.face[j];
        const FaceGeo<D> &F = fg[f];
        if (F.bc != 3) continue;  // uniform
        const FaceEq<D> &e = fe[f];
        double s[2 * NW + 2];
#pragma unroll
        for (int m = 0; m < 2 * NW + 2; ++m) s[m] = 0.0;
        for (int k = threadIdx.x; k < nv; k += BS) {
            double u[D], u2 = 0.0, un = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                u[d] = p.u[d * nv + k];
                u2 = fma(u[d], u[d], u2);
                un = fma(u[d], F.n[d], un);
            }
            const double wk = p.w[k];
            double I[2] = {0.0, 0.0};
            if (un > 0.0) {
                double fi[NC], gri[NC][D];
                limited_slope<D, FT>(gi, i, fin, nv, k, p.limiter, fi, gri);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    double v = fi[c], ug = 0.0;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        v = fma(gri[c][d], gi.dvec[j][d], v);
                        ug = fma(u[d], gri[c][d], ug);
                    }
                    I[c] = dt * v - 0.5 * dt * dt * ug;
                }
                s[2 * NW] = fma(wk * un, I[0], s[2 * NW]);
                double mm[NW];
#pragma unroll
                for (int m = 0; m < NW; ++m) mm[m] = 0.0;
                add_moments<D>(mm, wk * un, u, u2, I[0], NC > 1 ? I[NC - 1] : 0.0);
#pragma unroll
                for (int m = 0; m < NW; ++m) s[m] += mm[m];
            } else {
                const double H = dt * e.pref * gauss(j, (TENSOR ? (unsigned)p.kidx[k] : 0u), u, e.lam, e.U);
                I[0] = H;
                if constexpr (NC > 1) I[1] = e.bh * H;
                s[2 * NW + 1] = fma(wk * un, I[0], s[2 * NW + 1]);
                double mm[NW];
#pragma unroll
                for (int m = 0; m < NW; ++m) mm[m] = 0.0;
                add_moments<D>(mm, wk * un, u, u2, I[0], NC > 1 ? I[NC - 1] : 0.0);
#pragma unroll
                for (int m = 0; m < NW; ++m) s[NW + m] += mm[m];
            }
        }
        block_reduce<BS>(s, red, OpAdd{});
        const double rw = s[2 * NW + 1] != 0.0 ? -s[2 * NW] / s[2 * NW + 1] : 0.0;
#pragma unroll
        for (int jj = 0; jj < MF; ++jj)
            if (jj == j) rho_w[jj] = rw;
        if (threadIdx.x == 0 && p.wall_index) {
            const int widx = p.wall_index[f];
            if (widx >= 0)
#pragma unroll
                for (int m = 0; m < NW; ++m) p.wflux[(size_t)widx * NW + m] = (s[m] + rw * s[NW + m]) / dt;
        }
    }
}

// One colour's cells: cells[0..ncell) (stored indices), workgroups dealt to
// the XCDs in runs as for the gather sweep.  PF: the own stencil of the
// next velocity is loaded one iteration ahead.
template <int D, typename FT, int BS, bool TENSOR, bool PF>
__device__ __forceinline__ void push_cell(const Params p, int i, const FT *__restrict__ fin,
                                          typename AccOf<FT>::T *__restrict__ acc, int k0, int kn, int accv)
{
    using AT = typename AccOf<FT>::T;
    constexpr int NC = Dim<D>::NC, MF = Dim<D>::MF, NT = MF + 1;
    extern __shared__ double smem[];
    const int tid = threadIdx.x;
    const CellGeo<D> &gi = static_cast<const CellGeo<D> *>(p.cgeo)[i];
    const FaceGeo<D> *fg = static_cast<const FaceGeo<D> *>(p.fgeo);
    const FaceEq<D> *fe = static_cast<const FaceEq<D> *>(p.feq);
    const int nv = p.nv, nf = gi.nf, ntab = TENSOR ? p.ntab : 0;
    if constexpr (TENSOR) fill_tables<D, BS>(p, gi, to_prim<D>(p.W + (size_t)i * (D + 2)), smem);
    __syncthreads();
    const Gauss<D, TENSOR> gauss{smem, ntab, p.n1d[0], p.n1d[0] + p.n1d[1]};
    // wall densities of this cell's wall faces, from the step's wall kernel
    const double *rho_w = p.rho_w + (size_t)i * MF;

    // velocities [k0, k0 + kn); the accumulator holds accv velocities per
    // cell and component, starting at k0 (the whole set, or one chunk)
    const int kend = k0 + kn;
    const size_t base = (size_t)i * NC * accv;
    double pv0[NC], pvn[MF][NC];
    if (PF && k0 + tid < kend) load_stencil<D, FT>(gi, i, fin, nv, k0 + tid, pv0, pvn);
    for (int k = k0 + tid; k < kend; k += BS) {
        double v0[NC], vn[MF][NC];
        if constexpr (PF) {
#pragma unroll
            for (int m = 0; m < NC; ++m) {
                v0[m] = pv0[m];
#pragma unroll
                for (int j = 0; j < MF; ++j) vn[j][m] = pvn[j][m];
            }
            if (k + BS < kend) load_stencil<D, FT>(gi, i, fin, nv, k + BS, pv0, pvn);
        } else {
            load_stencil<D, FT>(gi, i, fin, nv, k, v0, vn);
        }
        double u[D], u2 = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            u[d] = p.u[d * nv + k];
            u2 = fma(u[d], u[d], u2);
        }
        const unsigned kx = TENSOR ? (unsigned)p.kidx[k] : 0u;
        double fi[NC], gri[NC][D];
        slope_from<D>(gi, p.limiter, v0, vn, fi, gri);
        double out[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c] = 0.0;
        // faces one at a time (not unrolled: their records are read with
        // scalar loads per face, which keeps the vector registers for the
        // velocities' values)
#pragma unroll 1
        for (int j = 0; j < nf; ++j) {
            const int f = gi.face[j];
            const FaceGeo<D> &F = fg[f];
            const FaceEq<D> &e = fe[f];
            double un = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) un = fma(u[d], F.n[d], un);
            const double uo = gi.side[j] ? -un : un;  // along this cell's outward normal
            if (F.bc == 0) {
                if (!(uo > 0.0)) continue;  // the neighbour is upwind: it adds this flux
                AT *an = acc + (size_t)gi.nb[j] * NC * accv;
                double val[NC], ug[NC], I[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    val[c] = fi[c];
                    ug[c] = 0.0;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        val[c] = fma(gri[c][d], gi.dvec[j][d], val[c]);
                        ug[c] = fma(u[d], gri[c][d], ug[c]);
                    }
                }
                const double H0 = e.pref * gauss(j, kx, u, e.lam, e.U);
                interface_integral<D>(e, u, u2, H0, val, ug, I);
                const double sa = F.area * uo;
                const double vn_inv = gi.nb_inv_vol[j];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const double fl = sa * I[c];
                    out[c] += fl;
                    // an atomic add without return: no load waits in the
                    // velocity loop (in a colour launch no other workgroup
                    // adds to this element, so the order of the sums stays
                    // fixed; the one-class unordered sweep gives that up)
                    unsafeAtomicAdd(an + (size_t)c * accv + (k - k0), from_f64<AT>(fl * vn_inv));
                }
            } else {
                double I[NC];
                if (un > 0.0) {
                    // outgoing through a wall or far-field face: free transport
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        double v = fi[c], ug = 0.0;
#pragma unroll
                        for (int d = 0; d < D; ++d) {
                            v = fma(gri[c][d], gi.dvec[j][d], v);
                            ug = fma(u[d], gri[c][d], ug);
                        }
                        I[c] = e.dt * v - e.hdt2 * ug;
                    }
                } else {
                    // incoming from the wall (density rho_w) or the ghost Maxwellian
                    const double H = (F.bc == 3 ? rho_w[j] : 1.0) * e.pref * gauss(j, kx, u, e.lam, e.U);
                    I[0] = e.dt * H;
                    if constexpr (NC > 1) I[1] = e.dt * e.bh * H;
                }
                const double sa = F.area * un;  // a boundary cell is the face's left cell
#pragma unroll
                for (int c = 0; c < NC; ++c) out[c] += sa * I[c];
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            AT *a = acc + base + (size_t)c * accv + (k - k0);
            unsafeAtomicAdd(a, from_f64<AT>(-out[c] * gi.inv_vol));
        }
    }
}

// The wall cells of a step (before the colours): wall densities per face slot
// into rho_w [cell][MF] and the wall flux of the step per wall face.
template <int D, typename FT, int BS, bool TENSOR>
__global__ __launch_bounds__(BS) void k_push_wall(Params p, const FT *__restrict__ fin, const int *__restrict__ cells,
                                                  int ncell)
{
    constexpr int MF = Dim<D>::MF, NT = MF + 1;
    extern __shared__ double smem[];
    if ((int)blockIdx.x >= ncell) return;
    const int i = cells[blockIdx.x];
    const CellGeo<D> &gi = static_cast<const CellGeo<D> *>(p.cgeo)[i];
    const int ntab = TENSOR ? p.ntab : 0;
    const CellStep<D> cs = cell_step<D>(p, i);
    if constexpr (TENSOR) fill_tables<D, BS>(p, gi, cs.pn, smem);
    __syncthreads();
    const Gauss<D, TENSOR> gauss{smem, ntab, p.n1d[0], p.n1d[0] + p.n1d[1]};
    double rho_w[MF];
    push_wall<D, FT, BS, TENSOR>(p, gi, i, fin, gauss, smem + NT * ntab, rho_w);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < MF; ++j) p.rho_w[(size_t)i * MF + j] = rho_w[j];
}

template <int D, typename FT, int BS, bool TENSOR>
__global__ __launch_bounds__(BS) void k_push(Params p, const FT *__restrict__ fin, typename AccOf<FT>::T *__restrict__ acc,
                                             const int *__restrict__ cells, int ncell, int k0, int kn, int accv,
                                             int ksplit)
{
    const int b = xcd_cell(blockIdx.x);
    if (b >= ncell) return;
    // this workgroup's share of [k0, k0 + kn): ksplit velocities from
    // k0 + blockIdx.y ksplit (the accumulator's velocity k0 is its column 0)
    const int ka = k0 + (int)blockIdx.y * ksplit, kb = min(k0 + kn, ka + ksplit);
    if (ka >= kb) return;
    push_cell<D, FT, BS, TENSOR, false>(p, cells[b], fin, acc + (ka - k0), ka, kb - ka, accv);
}

// (3D: held to 6 waves per SIMD, which fits without spills and measured 2 %
// faster than the 5 the compiler chooses; 2D would spill)
template <int D, typename FT, int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(D == 3 ? 6 : 1))) void k_push_pf(Params p, const FT *__restrict__ fin, typename AccOf<FT>::T *__restrict__ acc,
                                                const int *__restrict__ cells, int ncell, int k0, int kn, int accv,
                                                int ksplit)
{
    const int b = xcd_cell(blockIdx.x);
    if (b >= ncell) return;
    const int ka = k0 + (int)blockIdx.y * ksplit, kb = min(k0 + kn, ka + ksplit);
    if (ka >= kb) return;
    push_cell<D, FT, BS, true, true>(p, cells[b], fin, acc + (ka - k0), ka, kb - ka, accv);
}

// Velocity splits of a colour launch: a class of n cells gets up to enough
// workgroups to fill the chip (kPushFill), each with a share of the kn
// velocities that is a multiple of the workgroup size and at least
// kPushMinIters iterations long (every workgroup repeats the cell's set-up).
constexpr int kPushFill = 8192, kPushMinIters = 4;
inline int push_ksplit(int n, int kn, int bs)
{
    const int iters = (kn + bs - 1) / bs;  // velocity iterations of one workgroup
    const int split = std::max(1, std::min(iters / kPushMinIters, (kPushFill + n - 1) / n));
    const int per = (iters + split - 1) / split;
    return per * bs;
}

// After the last colour: W^{n+1}, tau^{n+1}, q^{n+1}, stage 2 into f and the
// next step's base into the accumulator; one wavefront per cell.
//   pass 1: moments of the stage-1 values h (and b) about U^n -- orders 0 to
//           3 of h, 0 and 1 of b -- in one sweep of the slab;
//   macro:  mass, momentum and energy from them -> W^{n+1}, tau^{n+1}; the
//           heat flux about U^{n+1} from the same moments, re-centred by
//           delta = U^{n+1} - U^n (exact algebra: the third-order moment of
//           (c - delta) expanded in delta), so no second pass is needed;
//   pass 2: stage 2 (Eq. microS2) into f, the base into acc (re-reading the
//           slab, which the cell's wavefront has just streamed through L2).
// V2: velocities in pairs, in the order of the base kernel.
template <int D> constexpr int sym_index(int a, int b)
{
    return a <= b ? a * D - a * (a - 1) / 2 + (b - a) : b * D - b * (b - 1) / 2 + (a - b);
}

template <int D, typename FT, bool TENSOR, bool V2>
__global__ __launch_bounds__(256) void k_push_final(Params p, FT *__restrict__ fout, typename AccOf<FT>::T *__restrict__ acc)
{
    using AT = typename AccOf<FT>::T;
    constexpr int NC = Dim<D>::NC, NW = D + 2, VW = V2 ? 2 : 1, NM = D * (D + 1) / 2;
    extern __shared__ double smem[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = kPushCellsPerGroup * xcd_cell(blockIdx.x) + wv;
    if (i >= p.nc) return;
    const int nv = p.nv;
    const double dt = p.dt, Pr = p.Pr;
    const size_t base = (size_t)i * NC * nv;
    double Wn[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) Wn[m] = p.W[(size_t)i * NW + m];
    const Prim<D> pn = to_prim<D>(Wn);

    // pass 1
    double m0 = 0.0, m1[D], m2[NM], m3[D], b0 = 0.0, b1[D];
#pragma unroll
    for (int d = 0; d < D; ++d) m1[d] = m3[d] = b1[d] = 0.0;
#pragma unroll
    for (int t = 0; t < NM; ++t) m2[t] = 0.0;
#pragma unroll 4
    for (int k0 = VW * lane; k0 < nv; k0 += VW * 64) {
        double v[VW][2];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if constexpr (V2)
                load2<AT>(acc + base + (size_t)c * nv + k0, v[0][c], v[1][c]);
            else
                v[0][c] = to_f64(acc[base + (size_t)c * nv + k0]);
        }
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const int k = k0 + e;
            const double w = p.w[k];
            double c[D], c2 = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                c[d] = p.u[d * nv + k] - pn.U[d];
                c2 = fma(c[d], c[d], c2);
            }
            const double wh = w * v[e][0];
            m0 += wh;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const double whc = wh * c[a];
                m1[a] += whc;
                m3[a] = fma(whc, c2, m3[a]);
#pragma unroll
                for (int bb = a; bb < D; ++bb) m2[sym_index<D>(a, bb)] = fma(whc, c[bb], m2[sym_index<D>(a, bb)]);
            }
            if constexpr (NC > 1) {
                const double wb = w * v[e][NC - 1];
                b0 += wb;
#pragma unroll
                for (int a = 0; a < D; ++a) b1[a] = fma(wb, c[a], b1[a]);
            }
        }
    }
    m0 = wave_sum(m0);
    b0 = wave_sum(b0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        m1[d] = wave_sum(m1[d]);
        m3[d] = wave_sum(m3[d]);
        b1[d] = wave_sum(b1[d]);
    }
#pragma unroll
    for (int t = 0; t < NM; ++t) m2[t] = wave_sum(m2[t]);

    // macro: mass, momentum, energy of the stage-1 values
    double mom[NW], trm2 = 0.0, um1 = 0.0, uu = 0.0;
    mom[0] = m0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        mom[1 + a] = fma(pn.U[a], m0, m1[a]);
        trm2 += m2[sym_index<D>(a, a)];
        um1 = fma(pn.U[a], m1[a], um1);
        uu = fma(pn.U[a], pn.U[a], uu);
    }
    mom[D + 1] = 0.5 * (trm2 + 2.0 * um1 + uu * m0 + b0);
    double W1[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) W1[m] = Wn[m] + (mom[m] - p.mom_part[(size_t)i * NW + m]);
    const Prim<D> p1 = to_prim<D>(W1);
    const double tau1 = collision_time(p1.rho, p1.lam, p.mu_ref, p.omega);
    // heat flux about U^{n+1}: sum w (c' |c'|^2 h + c' b) / 2 with c' = c - delta
    double dl[D], d2 = 0.0, m1d = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        dl[a] = p1.U[a] - pn.U[a];
        d2 = fma(dl[a], dl[a], d2);
        m1d = fma(m1[a], dl[a], m1d);
    }
    double q1[D];
    const double qden = 1.0 + Pr * dt / (2.0 * tau1);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double m2d = 0.0;
#pragma unroll
        for (int bb = 0; bb < D; ++bb) m2d = fma(m2[sym_index<D>(a, bb)], dl[bb], m2d);
        const double qa = m3[a] - 2.0 * m2d + d2 * m1[a] - dl[a] * trm2 + 2.0 * dl[a] * m1d - dl[a] * d2 * m0 + b1[a] -
                          dl[a] * b0;
        q1[a] = 0.5 * qa / qden;
    }

    double *tb = smem + (size_t)wv * (TENSOR ? p.ntab : 0);
    if constexpr (TENSOR) fill_wave_table<D>(p, p1.U, p1.lam, tb, lane);

    // pass 2: stage 2 into f, the next step's base into acc
    const double pref_1 = p1.rho * pow_lam_pi<D>(p1.lam);
    const double shk_1 = 4.0 * (1.0 - Pr) * p1.lam * p1.lam / (5.0 * p1.rho);
    const double a1 = 0.5 * dt / tau1, inv1 = 1.0 / (1.0 + a1);
    const double bh_1 = Dim<D>::M / (2.0 * p1.lam);
    double mb[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) mb[m] = 0.0;
#pragma unroll 2
    for (int k0 = VW * lane; k0 < nv; k0 += VW * 64) {
        double sv[VW][2];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if constexpr (V2)
                load2<AT>(acc + base + (size_t)c * nv + k0, sv[0][c], sv[1][c]);
            else
                sv[0][c] = to_f64(acc[base + (size_t)c * nv + k0]);
        }
        FT fo[VW][2];
        AT bo[VW][2];
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const int k = k0 + e;
            double u[D], u2;
            velocity<D>(p, k, u, u2);
            const unsigned kx = TENSOR ? (unsigned)p.kidx[k] : 0u;
            double fp[2];
            const double H = pref_1 * own_gauss<D, TENSOR>(p, tb, kx, u, p1.lam, p1.U);
            shakhov<D>(u, p1.U, p1.lam, shk_1, q1, bh_1, H, fp[0], fp[1]);
            double bv[2] = {0.0, 0.0};
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                fo[e][c] = from_f64<FT>((sv[e][c] + a1 * fp[c]) * inv1);
                // the base from f^{n+1} as stored (bitwise what the base
                // kernel computes from it after a restart)
                const double fd = opaque(to_f64(fo[e][c]));
                bo[e][c] = from_f64<AT>(fma(a1, fp[c] - fd, fd));
                bv[c] = to_f64(bo[e][c]);
            }
            add_moments<D>(mb, p.w[k], u, u2, bv[0], NC > 1 ? bv[NC - 1] : 0.0);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if constexpr (V2) {
                store2<FT>(fout + base + (size_t)c * nv + k0, fo[0][c], fo[1][c]);
                store2<AT>(acc + base + (size_t)c * nv + k0, bo[0][c], bo[1][c]);
            } else {
                fout[base + (size_t)c * nv + k0] = fo[0][c];
                acc[base + (size_t)c * nv + k0] = bo[0][c];
            }
        }
    }
#pragma unroll
    for (int m = 0; m < NW; ++m) mb[m] = wave_sum(mb[m]);
    if (lane == 0) {
        bool ok = p1.rho > 0.0 && p1.lam > 0.0 && isfinite(p1.rho) && isfinite(p1.lam);
#pragma unroll
        for (int m = 0; m < NW; ++m) {
            ok = ok && isfinite(W1[m]);
            p.W[(size_t)i * NW + m] = W1[m];
            const double dw = W1[m] - Wn[m];
            p.dW2[(size_t)i * NW + m] = dw * dw;
            p.mom_part[(size_t)i * NW + m] = mb[m];
        }
#pragma unroll
        for (int d = 0; d < D; ++d) p.q[(size_t)i * D + d] = q1[d];
        if (!ok) {
            atomicOr(p.err, 1);
            atomicMin(p.err + 1, i);
        }
    }
}

// ------------------------------------------------------------------------
// Surface quantities (Section 2.5): the macroscopic flux through each wall
// face in a step, from the f that started the step.  One workgroup per wall
// face: particles leaving the gas carry the limited reconstruction of f
// (free transport over the step), particles leaving the wall the wall
// Maxwellian of density rho_w; both sums are kept apart, rho_w follows from
// zero net mass flux, and F = (out + rho_w * in) / dt per unit area.
// ------------------------------------------------------------------------
template <int D, typename FT, int BS>
__global__ __launch_bounds__(BS) void k_wall_flux(Params p, const FT *__restrict__ fin,
                                                  const int *__restrict__ wall_faces, double *__restrict__ out)
{
    constexpr int NC = Dim<D>::NC, NW = D + 2;
    __shared__ double red[(BS / 64) * 2 * NW];
    const int f = wall_faces[blockIdx.x];
    const FaceGeo<D> &F = static_cast<const FaceGeo<D> *>(p.fgeo)[f];
    const FaceEq<D> &e = static_cast<const FaceEq<D> *>(p.feq)[f];
    const int i = F.l;
    const CellGeo<D> &gi = static_cast<const CellGeo<D> *>(p.cgeo)[i];
    int j = 0;
    for (int t = 0; t < gi.nf; ++t)
        if (gi.face[t] == f) j = t;
    const int nv = p.nv;
    const double dt = p.dt;
    double acc[2 * NW];
#pragma unroll
    for (int m = 0; m < 2 * NW; ++m) acc[m] = 0.0;
    for (int k = threadIdx.x; k < nv; k += BS) {
        double u[D], u2 = 0.0, un = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            u[d] = p.u[d * nv + k];
            u2 += u[d] * u[d];
            un += u[d] * F.n[d];
        }
        const double wk = p.w[k];
        double I[2] = {0.0, 0.0};
        int off = 0;
        if (un > 0.0) {
            double fi[NC], gri[NC][D];
            limited_slope<D, FT>(gi, i, fin, nv, k, p.limiter, fi, gri);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                double v = fi[c], ug = 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    v += gri[c][d] * gi.dvec[j][d];
                    ug += u[d] * gri[c][d];
                }
                I[c] = dt * v - 0.5 * dt * dt * ug;
            }
        } else {
            double c2 = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const double cd = u[d] - e.U[d];
                c2 += cd * cd;
            }
            const double H = e.pref * exp(-e.lam * c2);
            I[0] = dt * H;
            I[1] = NC > 1 ? dt * e.bh * H : 0.0;
            off = NW;
        }
        const double a = wk * un;
        double mom[NW];
        mom[0] = a * I[0];
#pragma unroll
        for (int d = 0; d < D; ++d) mom[1 + d] = a * u[d] * I[0];
        mom[NW - 1] = a * 0.5 * (u2 * I[0] + I[1]);
#pragma unroll
        for (int m = 0; m < NW; ++m) {
            acc[m] += off ? 0.0 : mom[m];
            acc[NW + m] += off ? mom[m] : 0.0;
        }
    }
    block_reduce<BS>(acc, red, OpAdd{});
    if (threadIdx.x == 0) {
        const double rho_w = acc[NW] != 0.0 ? -acc[0] / acc[NW] : 0.0;
#pragma unroll
        for (int m = 0; m < NW; ++m) out[(size_t)blockIdx.x * NW + m] = (acc[m] + rho_w * acc[NW + m]) / dt;
    }
}

// ------------------------------------------------------------------------
// L2 norm over cells of the last step's change of W (fixed order)
// ------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void residual(const Params p, double *out)
{
    constexpr int NW = D + 2;
    __shared__ double lds[4 * NW];
    double s[NW];
    for (int m = 0; m < NW; ++m) s[m] = 0.0;
    for (int i = threadIdx.x; i < p.nc; i += 256)
        for (int m = 0; m < NW; ++m) s[m] += p.dW2[(size_t)i * NW + m];
    block_reduce<256>(s, lds, OpAdd{});
    if (threadIdx.x == 0)
        for (int m = 0; m < NW; ++m) out[m] = sqrt(s[m]);
}

// One case: workgroup g sums the squared changes of a contiguous range of
// cells into part[g] (fixed order), then one workgroup sums the partial sums
// in order and takes the square roots.  Deterministic, and spread over the
// chip instead of one compute unit.
template <int D>
__global__ __launch_bounds__(256) void k_residual_part(Params p, double *part, int per)
{
    constexpr int NW = D + 2;
    __shared__ double lds[4 * NW];
    double s[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) s[m] = 0.0;
    const int i0 = blockIdx.x * per, i1 = min(p.nc, i0 + per);
    for (int i = i0 + threadIdx.x; i < i1; i += 256)
#pragma unroll
        for (int m = 0; m < NW; ++m) s[m] += p.dW2[(size_t)i * NW + m];
    block_reduce<256>(s, lds, OpAdd{});
    if (threadIdx.x == 0)
#pragma unroll
        for (int m = 0; m < NW; ++m) part[(size_t)blockIdx.x * NW + m] = s[m];
}

template <int D>
__global__ __launch_bounds__(256) void k_residual_final(const double *__restrict__ part, int ng, double *out)
{
    constexpr int NW = D + 2;
    __shared__ double lds[4 * NW];
    double s[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) s[m] = 0.0;
    for (int g = threadIdx.x; g < ng; g += 256)
#pragma unroll
        for (int m = 0; m < NW; ++m) s[m] += part[(size_t)g * NW + m];
    block_reduce<256>(s, lds, OpAdd{});
    if (threadIdx.x == 0)
#pragma unroll
        for (int m = 0; m < NW; ++m) out[m] = sqrt(s[m]);
}

// ------------------------------------------------------------------------
// Batched launches: the cases of a batch are laid end to end in one grid;
// off[c] is the first workgroup of case c.  Every workgroup finds its case
// by a binary search over off (wave-uniform, scalar) and runs the same
// per-cell or per-face code as the single-case kernels, on that case's
// parameters and buffers, so a case's result does not depend on the batch.
// ------------------------------------------------------------------------
// The descriptors are read-only for a launch: they are read through the
// constant address space, as kernel arguments are, so that the compiler may
// reload a case's parameters instead of holding them all in registers.
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(4))) BatchItem *ConstItems;
#else
typedef const BatchItem *ConstItems;  // the host pass only parses the kernels
#endif

__device__ __forceinline__ int batch_case(const int *__restrict__ off, int n, int b)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int D>
__global__ __launch_bounds__(256) void k_cell_grad_batch(const BatchItem *__restrict__ items, const int *__restrict__ off,
                                                         int n)
{
    const int c = batch_case(off, n, blockIdx.x);
    cell_grad<D>(((ConstItems)items)[c].p, (blockIdx.x - off[c]) * 256 + threadIdx.x);
}

template <int D>
__global__ __launch_bounds__(128) void k_face_eq_batch(const BatchItem *__restrict__ items, const int *__restrict__ off,
                                                       int n)
{
    const int c = batch_case(off, n, blockIdx.x);
    face_eq<D>(((ConstItems)items)[c].p, (blockIdx.x - off[c]) * 128 + threadIdx.x);
}

template <int D, typename FT, int BS, bool TENSOR, bool S1L>
__device__ __forceinline__ void sweep_batch(const BatchItem *__restrict__ items, const int *__restrict__ off, int n,
                                            int step)
{
    const int c = batch_case(off, n, blockIdx.x);
    ConstItems ci = (ConstItems)(items);
    const int cur = (ci[c].cur + step) & 1;
    sweep_cell<D, FT, BS, TENSOR, S1L, TENSOR>(ci[c].p, xcd_cell(blockIdx.x - off[c]),
                                               static_cast<const FT *>(ci[c].f[cur]),
                                               static_cast<FT *>(const_cast<void *>(ci[c].f[1 - cur])));
}
template <int D, typename FT, int BS, bool S1L>
__global__ __launch_bounds__(BS) void k_sweep_batch(const BatchItem *__restrict__ items, const int *__restrict__ off,
                                                    int n, int step)
{
    sweep_batch<D, FT, BS, false, S1L>(items, off, n, step);
}
template <int D, typename FT, int BS, bool S1L>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_sweep_batch_pf(
    const BatchItem *__restrict__ items, const int *__restrict__ off, int n, int step)
{
    sweep_batch<D, FT, BS, true, S1L>(items, off, n, step);
}

template <int D>
__global__ __launch_bounds__(256) void k_residual_batch(const BatchItem *__restrict__ items)
{
    ConstItems ci = (ConstItems)(items);
    residual<D>(ci[blockIdx.x].p, ci[blockIdx.x].res);
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
template <int D> hipError_t cfl_d(const Params &p, double *cell_dt, hipStream_t s)
{
    hipLaunchKernelGGL(k_cfl<D>, dim3(p.nc), dim3(256), 0, s, p, cell_dt);
    return hipGetLastError();
}
hipError_t launch_cfl(const Params &p, double *cell_dt, hipStream_t s)
{
    return p.dim == 2 ? cfl_d<2>(p, cell_dt, s) : cfl_d<3>(p, cell_dt, s);
}

template <int D, typename FT> hipError_t init_d(const Params &p, const double *prim0, void *f, hipStream_t s)
{
    hipLaunchKernelGGL((k_init<D, FT>), dim3(p.nc), dim3(256), 0, s, p, prim0, static_cast<FT *>(f));
    return hipGetLastError();
}
hipError_t launch_init(const Params &p, const double *prim0, void *f, hipStream_t s)
{
    if (p.dim == 2)
        return p.fstore == 2 ? init_d<2, bf16s>(p, prim0, f, s)
                             : (p.fstore ? init_d<2, float>(p, prim0, f, s) : init_d<2, double>(p, prim0, f, s));
    return p.fstore == 2 ? init_d<3, bf16s>(p, prim0, f, s)
                         : (p.fstore ? init_d<3, float>(p, prim0, f, s) : init_d<3, double>(p, prim0, f, s));
}

template <int D, typename FT> hipError_t moments_d(const Params &p, const void *f, hipStream_t s)
{
    hipLaunchKernelGGL((k_moments<D, FT>), dim3(p.nc), dim3(256), 0, s, p, static_cast<const FT *>(f));
    return hipGetLastError();
}
hipError_t launch_moments(const Params &p, const void *f, hipStream_t s)
{
    if (p.dim == 2)
        return p.fstore == 2 ? moments_d<2, bf16s>(p, f, s)
                             : (p.fstore ? moments_d<2, float>(p, f, s) : moments_d<2, double>(p, f, s));
    return p.fstore == 2 ? moments_d<3, bf16s>(p, f, s)
                         : (p.fstore ? moments_d<3, float>(p, f, s) : moments_d<3, double>(p, f, s));
}

template <int D> hipError_t prologue_d(const Params &p, hipStream_t s)
{
    hipLaunchKernelGGL(k_cell_grad<D>, dim3((p.nc + 255) / 256), dim3(256), 0, s, p);
    hipLaunchKernelGGL(k_face_eq<D>, dim3((p.nf + 127) / 128), dim3(128), 0, s, p);
    return hipGetLastError();
}
hipError_t launch_prologue(const Params &p, hipStream_t s)
{
    return p.dim == 2 ? prologue_d<2>(p, s) : prologue_d<3>(p, s);
}

// LDS a workgroup may take while four of them still fit on a CU (160 KB)
constexpr size_t kLdsPerWorkgroup = 40 * 1024;

size_t sweep_lds_bytes(const Params &p, bool *s1l)
{
    const int MF = p.dim == 2 ? Dim<2>::MF : Dim<3>::MF, NW = p.dim + 2, NC = p.dim == 2 ? Dim<2>::NC : Dim<3>::NC;
    const int NRED = NW > 2 * MF ? NW : 2 * MF;
    const size_t lds = sizeof(double) * ((size_t)(MF + 1) * (size_t)p.ntab + (256 / 64) * (size_t)NRED);
    const size_t fv = p.fstore == 2 ? 2 : (p.fstore == 1 ? 4 : 8);
    const size_t slab = fv * NC * (size_t)p.nv;
    *s1l = lds + slab <= kLdsPerWorkgroup;
    return *s1l ? lds + slab : lds;
}

int sweep_grid(int nc)
{
    constexpr int span = UGKS_XCDS * UGKS_XCD_RUN;
    return ((nc + span - 1) / span) * span;
}

template <int D, typename FT, int BS, bool TENSOR>
void sweep_launch(const Params &p, const void *fi, void *fo, hipStream_t s)
{
    bool s1l = false;
    const size_t lds = sweep_lds_bytes(p, &s1l);
    const unsigned grid = (unsigned)sweep_grid(p.nc);
    const FT *in = static_cast<const FT *>(fi);
    FT *out = static_cast<FT *>(fo);
    if constexpr (TENSOR) {
        if (s1l) hipLaunchKernelGGL((k_sweep_pf<D, FT, BS, true>), dim3(grid), dim3(BS), lds, s, p, in, out);
        else hipLaunchKernelGGL((k_sweep_pf<D, FT, BS, false>), dim3(grid), dim3(BS), lds, s, p, in, out);
    } else {
        if (s1l) hipLaunchKernelGGL((k_sweep<D, FT, BS, false, true>), dim3(grid), dim3(BS), lds, s, p, in, out);
        else hipLaunchKernelGGL((k_sweep<D, FT, BS, false, false>), dim3(grid), dim3(BS), lds, s, p, in, out);
    }
}

template <int D, typename FT> hipError_t sweep_d(const Params &p, const void *fi, void *fo, hipStream_t s)
{
    if (p.ntab > 0) sweep_launch<D, FT, 256, true>(p, fi, fo, s);
    else sweep_launch<D, FT, 256, false>(p, fi, fo, s);
    return hipGetLastError();
}
template <int D, typename FT, bool TENSOR> hipError_t inplace_d(const Params &p, void *fv, bool walls, hipStream_t s)
{
    constexpr int MF = Dim<D>::MF, NW = D + 2, NRED = (NW > 2 * MF) ? NW : 2 * MF;
    const size_t lds = sizeof(double) * ((size_t)(MF + 1) * (TENSOR ? p.ntab : 0) + (256 / 64) * NRED);
    const unsigned grid = (unsigned)sweep_grid(p.nc);
    FT *f = static_cast<FT *>(fv);
    if (walls) hipLaunchKernelGGL((k_wall_density<D, FT, 256, TENSOR>), dim3(grid), dim3(256), lds, s, p, f);
    for (int q = 0; q < p.nchunk; ++q) {
        const int c0 = q * p.chunk, cn = std::min(p.chunk, p.nv - c0);
        const int prev0 = (q - 1) * p.chunk, prevn = q > 0 ? p.chunk : 0;
        hipLaunchKernelGGL((k_sweep_chunk<D, FT, 256, TENSOR>), dim3(grid), dim3(256), lds, s, p, f, c0, cn, prev0,
                           prevn, q);
    }
    const int last0 = (p.nchunk - 1) * p.chunk;
    hipLaunchKernelGGL((k_sweep_finish<D, FT, 256, TENSOR>), dim3(grid), dim3(256), lds, s, p, f, last0,
                       p.nv - last0);
    return hipGetLastError();
}
template <int D, typename FT> hipError_t inplace_t(const Params &p, void *f, bool walls, hipStream_t s)
{
    return p.ntab > 0 ? inplace_d<D, FT, true>(p, f, walls, s) : inplace_d<D, FT, false>(p, f, walls, s);
}
hipError_t launch_sweep_inplace(const Params &p, void *f, bool walls, hipStream_t s)
{
    if (p.dim == 2)
        return p.fstore == 2 ? inplace_t<2, bf16s>(p, f, walls, s)
                             : (p.fstore ? inplace_t<2, float>(p, f, walls, s) : inplace_t<2, double>(p, f, walls, s));
    return p.fstore == 2 ? inplace_t<3, bf16s>(p, f, walls, s)
                         : (p.fstore ? inplace_t<3, float>(p, f, walls, s) : inplace_t<3, double>(p, f, walls, s));
}

hipError_t launch_sweep(const Params &p, const void *fi, void *fo, hipStream_t s)
{
    if (p.dim == 2)
        return p.fstore == 2 ? sweep_d<2, bf16s>(p, fi, fo, s)
                             : (p.fstore ? sweep_d<2, float>(p, fi, fo, s) : sweep_d<2, double>(p, fi, fo, s));
    return p.fstore == 2 ? sweep_d<3, bf16s>(p, fi, fo, s)
                         : (p.fstore ? sweep_d<3, float>(p, fi, fo, s) : sweep_d<3, double>(p, fi, fo, s));
}

// ------------------------------------------------------------------------
// Register-resident form of the push sweep's per-cell kernels, for slabs of
// at most NPT velocities per thread (one 256-thread workgroup per cell;
// thread t holds velocities t, t + 256, ...): the final kernel loads the
// whole stage-1 slab into registers in one go -- every load of a thread in
// flight together -- takes its moments, and applies stage 2 from the
// registers, so the slab is read once.  The base kernel of this form takes
// the velocities in the same order and reduces the same way.
// ------------------------------------------------------------------------
template <int D, int BS>
__device__ __forceinline__ void fill_group_table(const Params &p, double lam, double U0, double U1, double U2,
                                                 double *tb)
{
    for (int idx = threadIdx.x; idx < p.ntab; idx += BS) {
        const int ax = idx < p.n1d[0] ? 0 : (idx < p.n1d[0] + p.n1d[1] ? 1 : 2);
        const double Ud = ax == 0 ? U0 : (ax == 1 ? U1 : U2);
        const double c = p.u1d[idx] - Ud;
        tb[idx] = exp(-lam * c * c);
    }
    __syncthreads();
}

template <int D, typename FT, bool TENSOR>
__global__ __launch_bounds__(256) void k_push_base_r(Params p, const FT *__restrict__ fin, FT *__restrict__ acc)
{
    constexpr int NC = Dim<D>::NC, NW = D + 2, BS = 256;
    extern __shared__ double smem[];
    const int i = xcd_cell(blockIdx.x);
    if (i >= p.nc) return;
    const int nv = p.nv, tid = threadIdx.x;
    const CellStep<D> cs = cell_step<D>(p, i);
    double *tb = smem;
    double *red = smem + (TENSOR ? p.ntab : 0);
    if constexpr (TENSOR) fill_group_table<D, BS>(p, cs.pn.lam, cs.pn.U[0], cs.pn.U[1], cs.pn.U[D - 1], tb);
    const size_t base = (size_t)i * NC * nv;
    double mom[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) mom[m] = 0.0;
#pragma unroll 4
    for (int k = tid; k < nv; k += BS) {
        double u[D], u2;
        velocity<D>(p, k, u, u2);
        const unsigned kx = TENSOR ? (unsigned)p.kidx[k] : 0u;
        double fp[2];
        const double H = cs.pref_n * own_gauss<D, TENSOR>(p, tb, kx, u, cs.pn.lam, cs.pn.U);
        shakhov<D>(u, cs.pn.U, cs.pn.lam, cs.shk_n, cs.qn, cs.bh_n, H, fp[0], fp[1]);
        double bv[2] = {0.0, 0.0};
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double f = to_f64(fin[base + (size_t)c * nv + k]);
            const FT sv = from_f64<FT>(fma(cs.hdt_tau, fp[c] - f, f));
            acc[base + (size_t)c * nv + k] = sv;
            bv[c] = to_f64(sv);
        }
        add_moments<D>(mom, p.w[k], u, u2, bv[0], NC > 1 ? bv[NC - 1] : 0.0);
    }
    block_reduce_wide<BS>(mom, red, OpAdd{});
    if (tid == 0)
#pragma unroll
        for (int m = 0; m < NW; ++m) p.mom_part[(size_t)i * NW + m] = mom[m];
}

template <int D, typename FT, bool TENSOR, int NPT>
__global__ __launch_bounds__(256) void k_push_final_r(Params p, FT *__restrict__ fout, FT *__restrict__ acc)
{
    constexpr int NC = Dim<D>::NC, NW = D + 2, NM = D * (D + 1) / 2, BS = 256;
    // moments about U^n: m0, m1[D], m2[NM], m3[D], and for b: b0, b1[D]
    constexpr int NMOM = 1 + D + NM + D + (NC > 1 ? 1 + D : 0);
    extern __shared__ double smem[];
    const int i = xcd_cell(blockIdx.x);
    if (i >= p.nc) return;
    const int tid = threadIdx.x, nv = p.nv;
    const double dt = p.dt, Pr = p.Pr;
    const size_t base = (size_t)i * NC * nv;
    double *tb = smem;
    double *red = smem + (TENSOR ? p.ntab : 0);
    double Wn[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) Wn[m] = p.W[(size_t)i * NW + m];
    const Prim<D> pn = to_prim<D>(Wn);

    // pass 1: the slab into registers, in its storage precision (all loads
    // issued before any use)
    FT v[NPT][NC];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int k = tid + BS * j;
#pragma unroll
        for (int c = 0; c < NC; ++c) v[j][c] = k < nv ? acc[base + (size_t)c * nv + k] : from_f64<FT>(0.0);
    }
    double mm[NMOM];
#pragma unroll
    for (int t = 0; t < NMOM; ++t) mm[t] = 0.0;
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int k = tid + BS * j;
        if (k < nv) {
            const double w = p.w[k];
            double c[D], c2 = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                c[d] = p.u[d * nv + k] - pn.U[d];
                c2 = fma(c[d], c[d], c2);
            }
            const double wh = w * to_f64(v[j][0]);
            mm[0] += wh;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const double whc = wh * c[a];
                mm[1 + a] += whc;
                mm[1 + D + NM + a] = fma(whc, c2, mm[1 + D + NM + a]);
#pragma unroll
                for (int bb = a; bb < D; ++bb)
                    mm[1 + D + sym_index<D>(a, bb)] = fma(whc, c[bb], mm[1 + D + sym_index<D>(a, bb)]);
            }
            if constexpr (NC > 1) {
                const double wb = w * to_f64(v[j][NC - 1]);
                mm[1 + 2 * D + NM] += wb;
#pragma unroll
                for (int a = 0; a < D; ++a) mm[2 + 2 * D + NM + a] = fma(wb, c[a], mm[2 + 2 * D + NM + a]);
            }
        }
    }
    block_reduce_wide<BS>(mm, red, OpAdd{});
    const double m0 = mm[0];
    const double b0 = NC > 1 ? mm[1 + 2 * D + NM] : 0.0;
    double m1[D], m3[D], b1[D], m2[NM];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        m1[a] = mm[1 + a];
        m3[a] = mm[1 + D + NM + a];
        b1[a] = NC > 1 ? mm[2 + 2 * D + NM + a] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < NM; ++t) m2[t] = mm[1 + D + t];

    // macro: as in k_push_final (and macro_from_shift)
    double mom[NW], trm2 = 0.0, um1 = 0.0, uu = 0.0;
    mom[0] = m0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        mom[1 + a] = fma(pn.U[a], m0, m1[a]);
        trm2 += m2[sym_index<D>(a, a)];
        um1 = fma(pn.U[a], m1[a], um1);
        uu = fma(pn.U[a], pn.U[a], uu);
    }
    mom[D + 1] = 0.5 * (trm2 + 2.0 * um1 + uu * m0 + b0);
    double W1[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) W1[m] = Wn[m] + (mom[m] - p.mom_part[(size_t)i * NW + m]);
    const Prim<D> p1 = to_prim<D>(W1);
    const double tau1 = collision_time(p1.rho, p1.lam, p.mu_ref, p.omega);
    double dl[D], d2 = 0.0, m1d = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        dl[a] = p1.U[a] - pn.U[a];
        d2 = fma(dl[a], dl[a], d2);
        m1d = fma(m1[a], dl[a], m1d);
    }
    double q1[D];
    const double qden = 1.0 + Pr * dt / (2.0 * tau1);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double m2d = 0.0;
#pragma unroll
        for (int bb = 0; bb < D; ++bb) m2d = fma(m2[sym_index<D>(a, bb)], dl[bb], m2d);
        const double qa = m3[a] - 2.0 * m2d + d2 * m1[a] - dl[a] * trm2 + 2.0 * dl[a] * m1d - dl[a] * d2 * m0 + b1[a] -
                          dl[a] * b0;
        q1[a] = 0.5 * qa / qden;
    }
    if constexpr (TENSOR) fill_group_table<D, BS>(p, p1.lam, p1.U[0], p1.U[1], p1.U[D - 1], tb);

    // pass 2: stage 2 from the registers into f, the next base into acc
    const double pref_1 = p1.rho * pow_lam_pi<D>(p1.lam);
    const double shk_1 = 4.0 * (1.0 - Pr) * p1.lam * p1.lam / (5.0 * p1.rho);
    const double a1 = 0.5 * dt / tau1, inv1 = 1.0 / (1.0 + a1);
    const double bh_1 = Dim<D>::M / (2.0 * p1.lam);
    double mb[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) mb[m] = 0.0;
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int k = tid + BS * j;
        if (k < nv) {
            double u[D], u2;
            velocity<D>(p, k, u, u2);
            const unsigned kx = TENSOR ? (unsigned)p.kidx[k] : 0u;
            double fp[2];
            const double H = pref_1 * own_gauss<D, TENSOR>(p, tb, kx, u, p1.lam, p1.U);
            shakhov<D>(u, p1.U, p1.lam, shk_1, q1, bh_1, H, fp[0], fp[1]);
            double bv[2] = {0.0, 0.0};
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const FT fo = from_f64<FT>((to_f64(v[j][c]) + a1 * fp[c]) * inv1);
                fout[base + (size_t)c * nv + k] = fo;
                // the base from f^{n+1} as stored (bitwise what the base
                // kernel computes from it after a restart)
                const double fd = opaque(to_f64(fo));
                const FT bo = from_f64<FT>(fma(a1, fp[c] - fd, fd));
                acc[base + (size_t)c * nv + k] = bo;
                bv[c] = to_f64(bo);
            }
            add_moments<D>(mb, p.w[k], u, u2, bv[0], NC > 1 ? bv[NC - 1] : 0.0);
        }
    }
    block_reduce_wide<BS>(mb, red, OpAdd{});
    if (tid == 0) {
        bool ok = p1.rho > 0.0 && p1.lam > 0.0 && isfinite(p1.rho) && isfinite(p1.lam);
#pragma unroll
        for (int m = 0; m < NW; ++m) {
            ok = ok && isfinite(W1[m]);
            p.W[(size_t)i * NW + m] = W1[m];
            const double dw = W1[m] - Wn[m];
            p.dW2[(size_t)i * NW + m] = dw * dw;
            p.mom_part[(size_t)i * NW + m] = mb[m];
        }
#pragma unroll
        for (int d = 0; d < D; ++d) p.q[(size_t)i * D + d] = q1[d];
        if (!ok) {
            atomicOr(p.err, 1);
            atomicMin(p.err + 1, i);
        }
    }
}

// ------------------------------------------------------------------------
// Push sweep with one f buffer (the in-place mode).  The velocities are taken
// in chunks; per chunk, the base of the chunk's velocities goes into a ring of
// one chunk per cell (its moments added to the cell's running sum), the
// colour launches push the chunk's face fluxes into the ring, and the next
// turn kernel writes the stage-1 values back into f -- no later launch reads
// f^n at those velocities -- adding their moments about U^n (orders 0-3 of h,
// 0-1 of b) to a second running sum, before it fills the ring with the next
// chunk's base.  After the last chunk a final kernel forms
// W^{n+1}, tau^{n+1}, q^{n+1} from the two sums and applies stage 2 in place.
// The wall kernel runs first, while f still holds f^n at every velocity.
// ------------------------------------------------------------------------
template <int D> struct Shift {
    static constexpr int NC = Dim<D>::NC, NM = D * (D + 1) / 2;
    static constexpr int N = 1 + D + NM + D + (NC > 1 ? 1 + D : 0);
};

// one velocity's contribution to the moments about U^n (c = u - U^n)
template <int D>
__device__ __forceinline__ void add_shift_moments(double (&mm)[Shift<D>::N], double w, const double (&c)[D], double c2,
                                                  double h, double b)
{
    constexpr int NM = Shift<D>::NM;
    const double wh = w * h;
    mm[0] += wh;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double whc = wh * c[a];
        mm[1 + a] += whc;
        mm[1 + D + NM + a] = fma(whc, c2, mm[1 + D + NM + a]);
#pragma unroll
        for (int bb = a; bb < D; ++bb) mm[1 + D + sym_index<D>(a, bb)] = fma(whc, c[bb], mm[1 + D + sym_index<D>(a, bb)]);
    }
    if constexpr (Dim<D>::NC > 1) {
        const double wb = w * b;
        mm[1 + 2 * D + NM] += wb;
#pragma unroll
        for (int a = 0; a < D; ++a) mm[2 + 2 * D + NM + a] = fma(wb, c[a], mm[2 + 2 * D + NM + a]);
    }
}

// W^{n+1} (W^n + the stage-1 moments - the base's moments), its primitive
// state, tau^{n+1} and q^{n+1} (the re-centred heat flux of the stage-1
// values) from the moments about U^n
template <int D>
__device__ __forceinline__ void macro_from_shift(const Params &p, const double (&mm)[Shift<D>::N],
                                                 const double (&Wn)[D + 2], const Prim<D> &pn, const double *mom_base,
                                                 double (&W1)[D + 2], Prim<D> &p1, double &tau1, double (&q1)[D])
{
    constexpr int NW = D + 2, NM = Shift<D>::NM, NC = Dim<D>::NC;
    const double m0 = mm[0];
    const double b0 = NC > 1 ? mm[1 + 2 * D + NM] : 0.0;
    double m1[D], m3[D], b1[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        m1[a] = mm[1 + a];
        m3[a] = mm[1 + D + NM + a];
        b1[a] = NC > 1 ? mm[2 + 2 * D + NM + a] : 0.0;
    }
    double mom[NW], trm2 = 0.0, um1 = 0.0, uu = 0.0;
    mom[0] = m0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        mom[1 + a] = fma(pn.U[a], m0, m1[a]);
        trm2 += mm[1 + D + sym_index<D>(a, a)];
        um1 = fma(pn.U[a], m1[a], um1);
        uu = fma(pn.U[a], pn.U[a], uu);
    }
    mom[D + 1] = 0.5 * (trm2 + 2.0 * um1 + uu * m0 + b0);
#pragma unroll
    for (int m = 0; m < NW; ++m) W1[m] = Wn[m] + (mom[m] - mom_base[m]);
    p1 = to_prim<D>(W1);
    tau1 = collision_time(p1.rho, p1.lam, p.mu_ref, p.omega);
    double dl[D], d2 = 0.0, m1d = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        dl[a] = p1.U[a] - pn.U[a];
        d2 = fma(dl[a], dl[a], d2);
        m1d = fma(m1[a], dl[a], m1d);
    }
    const double qden = 1.0 + p.Pr * p.dt / (2.0 * tau1);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double m2d = 0.0;
#pragma unroll
        for (int bb = 0; bb < D; ++bb) m2d = fma(mm[1 + D + sym_index<D>(a, bb)], dl[bb], m2d);
        const double qa = m3[a] - 2.0 * m2d + d2 * m1[a] - dl[a] * trm2 + 2.0 * dl[a] * m1d - dl[a] * d2 * m0 + b1[a] -
                          dl[a] * b0;
        q1[a] = 0.5 * qa / qden;
    }
}

// The turn between two chunks, per cell: the previous chunk's stage-1
// values from the ring back into f, their moments about U^n added to mom_s;
// then the base of the next chunk's velocities into the ring, its moments
// added to mom_part (a chunk index of -1 skips that half; chunk 0 starts
// each sum).  Each cell's ring slice is touched only by its own workgroup.
template <int D, typename FT, bool TENSOR>
__global__ __launch_bounds__(256) void k_push_chunk_turn(Params p, FT *__restrict__ f,
                                                         typename AccOf<FT>::T *__restrict__ ring, int pc0, int pcn,
                                                         int pq, int nc0, int ncn, int nq)
{
    using AT = typename AccOf<FT>::T;
    constexpr int NC = Dim<D>::NC, NW = D + 2, BS = 256, N = Shift<D>::N;
    extern __shared__ double smem[];
    const int i = xcd_cell(blockIdx.x);
    if (i >= p.nc) return;
    const int nv = p.nv, ch = p.chunk, tid = threadIdx.x;
    const size_t fb = (size_t)i * NC * nv, rb = (size_t)i * NC * ch;
    double *tb = smem;
    double *red = smem + (TENSOR ? p.ntab : 0);
    const CellStep<D> cs = cell_step<D>(p, i);
    if (pq >= 0) {
        double mm[N];
#pragma unroll
        for (int t = 0; t < N; ++t) mm[t] = 0.0;
#pragma unroll 4
        for (int kk = tid; kk < pcn; kk += BS) {
            const int k = pc0 + kk;
            double v[2] = {0.0, 0.0};
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                // the moments are taken of the stage-1 value as summed (FP32
                // for bfloat16 f), as in the two-buffer final kernel
                const AT x = ring[rb + (size_t)c * ch + kk];
                if constexpr (sizeof(AT) == sizeof(FT))
                    f[fb + (size_t)c * nv + k] = x;
                else
                    f[fb + (size_t)c * nv + k] = from_f64<FT>(to_f64(x));
                v[c] = to_f64(x);
            }
            double cv[D], c2 = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                cv[d] = p.u[d * nv + k] - cs.pn.U[d];
                c2 = fma(cv[d], cv[d], c2);
            }
            add_shift_moments<D>(mm, p.w[k], cv, c2, v[0], NC > 1 ? v[NC - 1] : 0.0);
        }
        block_reduce_wide<BS>(mm, red, OpAdd{});
        if (tid == 0)
#pragma unroll
            for (int t = 0; t < N; ++t)
                p.mom_s[(size_t)i * N + t] = (pq == 0 ? 0.0 : p.mom_s[(size_t)i * N + t]) + mm[t];
    }
    if (nq >= 0) {
        if constexpr (TENSOR) fill_group_table<D, BS>(p, cs.pn.lam, cs.pn.U[0], cs.pn.U[1], cs.pn.U[D - 1], tb);
        double mom[NW];
#pragma unroll
        for (int m = 0; m < NW; ++m) mom[m] = 0.0;
#pragma unroll 2
        for (int kk = tid; kk < ncn; kk += BS) {
            const int k = nc0 + kk;
            double u[D], u2;
            velocity<D>(p, k, u, u2);
            const unsigned kx = TENSOR ? (unsigned)p.kidx[k] : 0u;
            double fp[2];
            const double H = cs.pref_n * own_gauss<D, TENSOR>(p, tb, kx, u, cs.pn.lam, cs.pn.U);
            shakhov<D>(u, cs.pn.U, cs.pn.lam, cs.shk_n, cs.qn, cs.bh_n, H, fp[0], fp[1]);
            double bv[2] = {0.0, 0.0};
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double fv = to_f64(f[fb + (size_t)c * nv + k]);
                const AT sv = from_f64<AT>(fma(cs.hdt_tau, fp[c] - fv, fv));
                ring[rb + (size_t)c * ch + kk] = sv;
                bv[c] = to_f64(sv);
            }
            add_moments<D>(mom, p.w[k], u, u2, bv[0], NC > 1 ? bv[NC - 1] : 0.0);
        }
        block_reduce_wide<BS>(mom, red, OpAdd{});
        if (tid == 0)
#pragma unroll
            for (int m = 0; m < NW; ++m)
                p.mom_part[(size_t)i * NW + m] = (nq == 0 ? 0.0 : p.mom_part[(size_t)i * NW + m]) + mom[m];
    }
}

// after the last chunk: W^{n+1}, tau^{n+1}, q^{n+1}, stage 2 in place
template <int D, typename FT, bool TENSOR>
__global__ __launch_bounds__(256) void k_push_final_inplace(Params p, FT *__restrict__ f)
{
    constexpr int NC = Dim<D>::NC, NW = D + 2, BS = 256, N = Shift<D>::N;
    extern __shared__ double smem[];
    const int i = xcd_cell(blockIdx.x);
    if (i >= p.nc) return;
    const int nv = p.nv, tid = threadIdx.x;
    const double dt = p.dt, Pr = p.Pr;
    double Wn[NW];
#pragma unroll
    for (int m = 0; m < NW; ++m) Wn[m] = p.W[(size_t)i * NW + m];
    const Prim<D> pn = to_prim<D>(Wn);
    double mm[N];
#pragma unroll
    for (int t = 0; t < N; ++t) mm[t] = p.mom_s[(size_t)i * N + t];
    double W1[NW], tau1, q1[D];
    Prim<D> p1;
    macro_from_shift<D>(p, mm, Wn, pn, p.mom_part + (size_t)i * NW, W1, p1, tau1, q1);
    double *tb = smem;
    if constexpr (TENSOR) fill_group_table<D, BS>(p, p1.lam, p1.U[0], p1.U[1], p1.U[D - 1], tb);
    const double pref_1 = p1.rho * pow_lam_pi<D>(p1.lam);
    const double shk_1 = 4.0 * (1.0 - Pr) * p1.lam * p1.lam / (5.0 * p1.rho);
    const double a1 = 0.5 * dt / tau1, inv1 = 1.0 / (1.0 + a1);
    const double bh_1 = Dim<D>::M / (2.0 * p1.lam);
    const size_t fb = (size_t)i * NC * nv;
#pragma unroll 2
    for (int k = tid; k < nv; k += BS) {
        double u[D], u2;
        velocity<D>(p, k, u, u2);
        const unsigned kx = TENSOR ? (unsigned)p.kidx[k] : 0u;
        double fp[2];
        const double H = pref_1 * own_gauss<D, TENSOR>(p, tb, kx, u, p1.lam, p1.U);
        shakhov<D>(u, p1.U, p1.lam, shk_1, q1, bh_1, H, fp[0], fp[1]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            FT *q = f + fb + (size_t)c * nv + k;
            *q = from_f64<FT>((to_f64(*q) + a1 * fp[c]) * inv1);
        }
    }
    if (tid == 0) {
        bool ok = p1.rho > 0.0 && p1.lam > 0.0 && isfinite(p1.rho) && isfinite(p1.lam);
#pragma unroll
        for (int m = 0; m < NW; ++m) {
            ok = ok && isfinite(W1[m]);
            p.W[(size_t)i * NW + m] = W1[m];
            const double dw = W1[m] - Wn[m];
            p.dW2[(size_t)i * NW + m] = dw * dw;
        }
#pragma unroll
        for (int d = 0; d < D; ++d) p.q[(size_t)i * D + d] = q1[d];
        if (!ok) {
            atomicOr(p.err, 1);
            atomicMin(p.err + 1, i);
        }
    }
}

// ------------------------------------------------------------------------
// push sweep launches: the stage-1 base (when stale), the wall cells, one
// launch per colour (split over velocities when small), the final kernel
// ------------------------------------------------------------------------
template <int D, typename FT, bool TENSOR>
hipError_t push_t(const Params &p, void *fv, void *av, bool need_base, const int *cells, const int *coff, int ncol,
                  const int *wall_cells, int n_wall_cells, hipStream_t s)
{
    constexpr int MF = Dim<D>::MF, NW = D + 2, NC = Dim<D>::NC, BS = 256;
    using AT = typename AccOf<FT>::T;
    const FT *fin = static_cast<const FT *>(fv);
    FT *f = static_cast<FT *>(fv);
    AT *acc = static_cast<AT *>(av);
    const size_t tab = sizeof(double) * (size_t)(MF + 1) * (TENSOR ? p.ntab : 0);
    const size_t red = sizeof(double) * ((BS / 64) * (2 * NW + 2) + MF);
    const unsigned gc = (unsigned)sweep_grid(p.nc);
    // the per-cell streaming kernels: a wavefront per cell, four per group;
    // velocity pairs when the count is even (every slab offset is then
    // even: aligned 2-wide accesses)
    const unsigned gw = (unsigned)sweep_grid((p.nc + kPushCellsPerGroup - 1) / kPushCellsPerGroup);
    const size_t ltab = sizeof(double) * (size_t)kPushCellsPerGroup * (TENSOR ? p.ntab : 0);
    const bool v2 = p.nv % 2 == 0;
    // the register-resident form for FP64 f where a thread's share of the
    // slab fits in 48 registers (n_comp x NPT values; with FP32 f it measured
    // slower than the wavefront form)
    const int npt = (p.nv + 255) / 256;
    const int slab_regs = NC * 2;
    int reg_form = 0;
    if (sizeof(FT) == 8) {
        if (npt <= 12 && 12 * slab_regs <= 48) reg_form = 12;
        else if (npt <= 18 && 18 * slab_regs <= 48) reg_form = 18;
        else if (npt <= 24 && 24 * slab_regs <= 48) reg_form = 24;
    }
    const size_t lreg = sizeof(double) * ((TENSOR ? (size_t)p.ntab : 0) + 5 * 16);
    if (need_base && reg_form) {
        if constexpr (sizeof(FT) == 8)
            hipLaunchKernelGGL((k_push_base_r<D, FT, TENSOR>), dim3(gc), dim3(256), lreg, s, p, fin, acc);
    } else if (need_base) {
        if (v2)
            hipLaunchKernelGGL((k_push_base<D, FT, TENSOR, true>), dim3(gw), dim3(256), ltab, s, p, fin, acc);
        else
            hipLaunchKernelGGL((k_push_base<D, FT, TENSOR, false>), dim3(gw), dim3(256), ltab, s, p, fin, acc);
    }
    if (n_wall_cells > 0)
        hipLaunchKernelGGL((k_push_wall<D, FT, BS, TENSOR>), dim3(n_wall_cells), dim3(BS), tab + red, s, p, fin,
                           wall_cells, n_wall_cells);
    for (int c = 0; c < ncol; ++c) {
        const int n = coff[c + 1] - coff[c];
        if (n <= 0) continue;
        const unsigned g = (unsigned)sweep_grid(n);
        const int ks = push_ksplit(n, p.nv, BS);
        const dim3 grid(g, (unsigned)((p.nv + ks - 1) / ks));
        if constexpr (TENSOR)
            hipLaunchKernelGGL((k_push_pf<D, FT, BS>), grid, dim3(BS), tab + red, s, p, fin, acc, cells + coff[c], n, 0,
                               p.nv, p.nv, ks);
        else
            hipLaunchKernelGGL((k_push<D, FT, BS, false>), grid, dim3(BS), tab + red, s, p, fin, acc, cells + coff[c],
                               n, 0, p.nv, p.nv, ks);
    }
    if (reg_form) {
        if constexpr (sizeof(FT) == 8) {
            if (reg_form == 12)
                hipLaunchKernelGGL((k_push_final_r<D, FT, TENSOR, 12>), dim3(gc), dim3(256), lreg, s, p, f, acc);
            else if (reg_form == 18)
                hipLaunchKernelGGL((k_push_final_r<D, FT, TENSOR, 18>), dim3(gc), dim3(256), lreg, s, p, f, acc);
            else
                hipLaunchKernelGGL((k_push_final_r<D, FT, TENSOR, 24>), dim3(gc), dim3(256), lreg, s, p, f, acc);
        }
    } else if (v2)
        hipLaunchKernelGGL((k_push_final<D, FT, TENSOR, true>), dim3(gw), dim3(256), ltab, s, p, f, acc);
    else
        hipLaunchKernelGGL((k_push_final<D, FT, TENSOR, false>), dim3(gw), dim3(256), ltab, s, p, f, acc);
    return hipGetLastError();
}

template <int D, typename FT>
hipError_t push_d(const Params &p, void *f, void *acc, bool need_base, const int *cells, const int *coff, int ncol,
                  const int *wc, int nwc, hipStream_t s)
{
    return p.ntab > 0 ? push_t<D, FT, true>(p, f, acc, need_base, cells, coff, ncol, wc, nwc, s)
                      : push_t<D, FT, false>(p, f, acc, need_base, cells, coff, ncol, wc, nwc, s);
}

template <int D, typename FT, bool TENSOR>
hipError_t push_inplace_t(const Params &p, void *fv, const int *cells, const int *coff, int ncol,
                          const int *wall_cells, int n_wall_cells, hipStream_t s)
{
    constexpr int MF = Dim<D>::MF, NW = D + 2, BS = 256;
    using AT = typename AccOf<FT>::T;
    FT *f = static_cast<FT *>(fv);
    AT *ring = static_cast<AT *>(p.ring);
    const size_t tab = sizeof(double) * (size_t)(MF + 1) * (TENSOR ? p.ntab : 0);
    const size_t red = sizeof(double) * ((BS / 64) * (2 * NW + 2) + MF);
    const unsigned gc = (unsigned)sweep_grid(p.nc);
    const size_t lcell = sizeof(double) * ((TENSOR ? (size_t)p.ntab : 0) + 5 * 16);
    if (n_wall_cells > 0)
        hipLaunchKernelGGL((k_push_wall<D, FT, BS, TENSOR>), dim3(n_wall_cells), dim3(BS), tab + red, s, p, f,
                           wall_cells, n_wall_cells);
    for (int q = 0; q < p.nchunk; ++q) {
        const int c0 = q * p.chunk, cn = std::min(p.chunk, p.nv - c0);
        // the previous chunk back into f, this chunk's base into the ring
        const int pc0 = (q - 1) * p.chunk;
        hipLaunchKernelGGL((k_push_chunk_turn<D, FT, TENSOR>), dim3(gc), dim3(BS), lcell, s, p, f, ring, pc0,
                           q > 0 ? p.chunk : 0, q - 1, c0, cn, q);
        for (int c = 0; c < ncol; ++c) {
            const int n = coff[c + 1] - coff[c];
            if (n <= 0) continue;
            const unsigned g = (unsigned)sweep_grid(n);
            const int ks = push_ksplit(n, cn, BS);
            const dim3 grid(g, (unsigned)((cn + ks - 1) / ks));
            if constexpr (TENSOR)
                hipLaunchKernelGGL((k_push_pf<D, FT, BS>), grid, dim3(BS), tab + red, s, p, f, ring, cells + coff[c], n,
                                   c0, cn, p.chunk, ks);
            else
                hipLaunchKernelGGL((k_push<D, FT, BS, false>), grid, dim3(BS), tab + red, s, p, f, ring,
                                   cells + coff[c], n, c0, cn, p.chunk, ks);
        }
    }
    {
        const int q = p.nchunk - 1, c0 = q * p.chunk;
        hipLaunchKernelGGL((k_push_chunk_turn<D, FT, TENSOR>), dim3(gc), dim3(BS), lcell, s, p, f, ring, c0,
                           p.nv - c0, q, 0, 0, -1);
    }
    hipLaunchKernelGGL((k_push_final_inplace<D, FT, TENSOR>), dim3(gc), dim3(BS), lcell, s, p, f);
    return hipGetLastError();
}

template <int D, typename FT>
hipError_t push_inplace_d(const Params &p, void *f, const int *cells, const int *coff, int ncol, const int *wc,
                          int nwc, hipStream_t s)
{
    return p.ntab > 0 ? push_inplace_t<D, FT, true>(p, f, cells, coff, ncol, wc, nwc, s)
                      : push_inplace_t<D, FT, false>(p, f, cells, coff, ncol, wc, nwc, s);
}

hipError_t launch_push_inplace(const Params &p, void *f, const int *cells, const int *coff, int ncol,
                               const int *wall_cells, int n_wall_cells, hipStream_t s)
{
    // bfloat16 f: the ring holds FP32 stage-1 sums
    if (p.dim == 2)
        return p.fstore == 2 ? push_inplace_d<2, bf16s>(p, f, cells, coff, ncol, wall_cells, n_wall_cells, s)
               : p.fstore    ? push_inplace_d<2, float>(p, f, cells, coff, ncol, wall_cells, n_wall_cells, s)
                             : push_inplace_d<2, double>(p, f, cells, coff, ncol, wall_cells, n_wall_cells, s);
    return p.fstore == 2 ? push_inplace_d<3, bf16s>(p, f, cells, coff, ncol, wall_cells, n_wall_cells, s)
           : p.fstore    ? push_inplace_d<3, float>(p, f, cells, coff, ncol, wall_cells, n_wall_cells, s)
                         : push_inplace_d<3, double>(p, f, cells, coff, ncol, wall_cells, n_wall_cells, s);
}

hipError_t launch_push_step(const Params &p, void *f, void *acc, bool need_base, const int *cells, const int *coff,
                            int ncol, const int *wall_cells, int n_wall_cells, hipStream_t s)
{
    // bfloat16 f: acc holds FP32 stage-1 sums
    if (p.dim == 2)
        return p.fstore == 2 ? push_d<2, bf16s>(p, f, acc, need_base, cells, coff, ncol, wall_cells, n_wall_cells, s)
               : p.fstore    ? push_d<2, float>(p, f, acc, need_base, cells, coff, ncol, wall_cells, n_wall_cells, s)
                             : push_d<2, double>(p, f, acc, need_base, cells, coff, ncol, wall_cells, n_wall_cells, s);
    return p.fstore == 2 ? push_d<3, bf16s>(p, f, acc, need_base, cells, coff, ncol, wall_cells, n_wall_cells, s)
           : p.fstore    ? push_d<3, float>(p, f, acc, need_base, cells, coff, ncol, wall_cells, n_wall_cells, s)
                         : push_d<3, double>(p, f, acc, need_base, cells, coff, ncol, wall_cells, n_wall_cells, s);
}

// Surface quantities of Section 2.5 from the wall flux of the last step (per
// unit area and time), one thread per wall face: surface pressure
// p_w = F_m . n (n out of the gas), shear stress sigma_w = |F_m - p_w n|,
// heat flux q_w = the energy component, and the coefficients of
// Section 4.1: Cp = p_w / d, Ct = sigma_w / d, Ch = q_w / (d u_inf) with
// d = rho_inf u_inf^2 / 2.  out [n][6].
template <int D>
__global__ __launch_bounds__(256) void k_surface(Params p, const int *__restrict__ wall_faces,
                                                 const double *__restrict__ flux, int n, double rho_inf, double u_inf,
                                                 double *__restrict__ out)
{
    constexpr int NW = D + 2;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    const FaceGeo<D> &F = static_cast<const FaceGeo<D> *>(p.fgeo)[wall_faces[t]];
    const double *w = flux + (size_t)t * NW;
    double pw = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) pw += w[1 + d] * F.n[d];
    double s2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double tang = w[1 + d] - pw * F.n[d];
        s2 += tang * tang;
    }
    const double sig = sqrt(s2), qw = w[NW - 1];
    const double dyn = 0.5 * rho_inf * u_inf * u_inf;
    double *o = out + (size_t)t * 6;
    o[0] = pw;
    o[1] = sig;
    o[2] = qw;
    o[3] = pw / dyn;
    o[4] = sig / dyn;
    o[5] = qw / (dyn * u_inf);
}

hipError_t launch_surface(const Params &p, const int *faces, const double *flux, int n, double rho_inf, double u_inf,
                          double *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const dim3 grid((n + 255) / 256);
    if (p.dim == 2) hipLaunchKernelGGL(k_surface<2>, grid, dim3(256), 0, s, p, faces, flux, n, rho_inf, u_inf, out);
    else hipLaunchKernelGGL(k_surface<3>, grid, dim3(256), 0, s, p, faces, flux, n, rho_inf, u_inf, out);
    return hipGetLastError();
}

template <int D, typename FT>
hipError_t wall_flux_d(const Params &p, const void *f, const int *faces, int n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL((k_wall_flux<D, FT, 256>), dim3(n), dim3(256), 0, s, p, static_cast<const FT *>(f), faces, out);
    return hipGetLastError();
}
hipError_t launch_wall_flux(const Params &p, const void *f, const int *faces, int n, double *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (p.dim == 2)
        return p.fstore == 2 ? wall_flux_d<2, bf16s>(p, f, faces, n, out, s)
                             : (p.fstore ? wall_flux_d<2, float>(p, f, faces, n, out, s)
                                         : wall_flux_d<2, double>(p, f, faces, n, out, s));
    return p.fstore == 2 ? wall_flux_d<3, bf16s>(p, f, faces, n, out, s)
                         : (p.fstore ? wall_flux_d<3, float>(p, f, faces, n, out, s)
                                     : wall_flux_d<3, double>(p, f, faces, n, out, s));
}

hipError_t launch_batch_prologue(const BatchItem *items, int n, const int *off_grad, int grid_grad,
                                 const int *off_face, int grid_face, int dim, hipStream_t s)
{
    if (dim == 2) {
        hipLaunchKernelGGL(k_cell_grad_batch<2>, dim3(grid_grad), dim3(256), 0, s, items, off_grad, n);
        hipLaunchKernelGGL(k_face_eq_batch<2>, dim3(grid_face), dim3(128), 0, s, items, off_face, n);
    } else {
        hipLaunchKernelGGL(k_cell_grad_batch<3>, dim3(grid_grad), dim3(256), 0, s, items, off_grad, n);
        hipLaunchKernelGGL(k_face_eq_batch<3>, dim3(grid_face), dim3(128), 0, s, items, off_face, n);
    }
    return hipGetLastError();
}

template <int D, typename FT, bool TENSOR>
void batch_sweep_t(const BatchItem *items, int n, const int *off, int grid, int step, bool s1l, size_t lds, hipStream_t s)
{
    if constexpr (TENSOR) {
        if (s1l) hipLaunchKernelGGL((k_sweep_batch_pf<D, FT, 256, true>), dim3(grid), dim3(256), lds, s, items, off, n, step);
        else hipLaunchKernelGGL((k_sweep_batch_pf<D, FT, 256, false>), dim3(grid), dim3(256), lds, s, items, off, n, step);
    } else {
        if (s1l) hipLaunchKernelGGL((k_sweep_batch<D, FT, 256, true>), dim3(grid), dim3(256), lds, s, items, off, n, step);
        else hipLaunchKernelGGL((k_sweep_batch<D, FT, 256, false>), dim3(grid), dim3(256), lds, s, items, off, n, step);
    }
}
template <int D, typename FT>
void batch_sweep_f(const BatchItem *items, int n, const int *off, int grid, int step, bool tensor, bool s1l, size_t lds,
                   hipStream_t s)
{
    if (tensor) batch_sweep_t<D, FT, true>(items, n, off, grid, step, s1l, lds, s);
    else batch_sweep_t<D, FT, false>(items, n, off, grid, step, s1l, lds, s);
}
template <int D>
void batch_sweep_d(const BatchItem *items, int n, const int *off, int grid, int step, int fstore, bool tensor, bool s1l,
                   size_t lds, hipStream_t s)
{
    if (fstore == 2) batch_sweep_f<D, bf16s>(items, n, off, grid, step, tensor, s1l, lds, s);
    else if (fstore == 1) batch_sweep_f<D, float>(items, n, off, grid, step, tensor, s1l, lds, s);
    else batch_sweep_f<D, double>(items, n, off, grid, step, tensor, s1l, lds, s);
}
hipError_t launch_batch_sweep(const BatchItem *items, int n, const int *off, int grid, int step, int dim, int fstore,
                              bool tensor, bool s1l, size_t lds, hipStream_t s)
{
    if (dim == 2) batch_sweep_d<2>(items, n, off, grid, step, fstore, tensor, s1l, lds, s);
    else batch_sweep_d<3>(items, n, off, grid, step, fstore, tensor, s1l, lds, s);
    return hipGetLastError();
}

hipError_t launch_batch_residual(const BatchItem *items, int n, int dim, hipStream_t s)
{
    if (dim == 2) hipLaunchKernelGGL(k_residual_batch<2>, dim3(n), dim3(256), 0, s, items);
    else hipLaunchKernelGGL(k_residual_batch<3>, dim3(n), dim3(256), 0, s, items);
    return hipGetLastError();
}

int residual_groups(int nc) { return std::max(1, std::min(kResidualGroups, (nc + 2047) / 2048)); }

// ------------------------------------------------------------------------
// Fixed device scratch of the allocation-free batched step: the batch
// descriptors and offset tables.  Each GPU holds its own copy until the
// process ends.  In host code `scratch` names a host-side stand-in, not a
// device address: the device address is looked up once per device, with that
// device current, and only that address is ever handed to copies or kernels.
// ------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_residual(const Params &p, double *out, hipStream_t s)
{
    const int ng = residual_groups(p.nc), per = (p.nc + ng - 1) / ng;
    double *part = out + (p.dim + 2);
    if (p.dim == 2) {
        hipLaunchKernelGGL(k_residual_part<2>, dim3(ng), dim3(256), 0, s, p, part, per);
        hipLaunchKernelGGL(k_residual_final<2>, dim3(1), dim3(256), 0, s, part, ng, out);
    } else {
        hipLaunchKernelGGL(k_residual_part<3>, dim3(ng), dim3(256), 0, s, p, part, per);
        hipLaunchKernelGGL(k_residual_final<3>, dim3(1), dim3(256), 0, s, part, ng, out);
    }
    return hipGetLastError();
}

}  // namespace ugx
