// sme_step_common.h -- device helpers shared by the step kernels.
//
// One launch per time step does the whole step for every cell:
//   hyperbolic predictor  Q* = Q^n - dt/|V| sum_f |e_f| (Fhat_f + D_f / 2)   (Eq. (3a))
//   friction ODE          Q^{n+1} = Q* + dt S(Q*)                           (Eq. (3d))
//   CFL ratio of Q^{n+1}  r_i = sum_f |e_f| lam(Q_i, n_f) / (2 |V_i|), max-reduced
// and the next launch reads dt = CFL / max r from the device (Sec. 3.1: adaptive
// step), so a run needs no host round trip.
//
// Layouts: SoA FP64 state q[f * stride + cell].
//   1D and structured 2D: a 64-lane wavefront owns 64 consecutive columns
//   (62 outputs + one halo column each side).  Each lane computes the x-face to
//   its right once; the left cell's share travels one lane up through a
//   cross-lane shuffle.  In 2D the wave then marches up a strip of `rows` rows,
//   keeping the previous row in registers, so every y-face is computed once too.
//   Triangles: one lane per cell in a bandwidth-reducing (RCM) order, three
//   neighbour gathers; each face is evaluated in a canonical orientation (from
//   the lower to the higher cell index) so both neighbours see bitwise equal
//   face values.
// All reductions are wave shuffles plus one unsigned 64-bit atomic max per
// wave on the bit pattern of a non-negative double: exact and order-free, so
// runs are bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>

#include "sme_kernels.h"

namespace sme {
namespace detail {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kOut = kWave - 2;  // outputs per wave along x
constexpr int kXcd = 8;          // compute dies (XCDs) of the MI355X, each with its own L2

__device__ __forceinline__ double step_dt(const StepArgs &a)
{
    const Slot &sl = a.slots[a.sa];
    double dt;
    if (a.dt_fixed > 0.0) {
        dt = a.dt_fixed;
    } else {
        const double r = slot_ratio(sl);
        dt = r > 0.0 ? a.cfl / r : 0.0;
    }
    if (a.t_end > 0.0) dt = fmin(dt, fmax(a.t_end - sl.t, 0.0));
    return dt;
}

// bookkeeping of the time slots, done by one lane of the grid
__device__ __forceinline__ void slot_update(const StepArgs &a, double dt)
{
    const Slot &sl = a.slots[a.sa];
    Slot &nx = a.slots[a.sb];
    nx.t = sl.t + dt;
    nx.dt = dt;
    nx.step = sl.step + (dt > 0.0 ? 1 : 0);
#pragma unroll
    for (int w = 0; w < kRatioWords; ++w) a.slots[a.sc].r[w].bits = 0ull;
    a.slots[a.sc].lbits = 0ull;
}

// A step past the end time (dt = 0) leaves the state as it is: every thread of
// the grid copies its share of Q^n to Q^{n+1}, and one lane carries the CFL
// ratio and largest wave speed over to the next slot (no block reduces).
// dt is the same for the whole grid, so either every block takes this path
// or none does.
__device__ __forceinline__ void noop_step(const StepArgs &a, int nf)
{
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int f = 0; f < nf; ++f)
        for (int64_t i = t0; i < a.ncells; i += nth) a.qn[f * a.stride + i] = a.q[f * a.stride + i];
    if (t0 == 0) {
#pragma unroll
        for (int w = 0; w < kRatioWords; ++w) a.slots[a.sb].r[w].bits = a.slots[a.sa].r[w].bits;
        a.slots[a.sb].lbits = a.slots[a.sa].lbits;
    }
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
}

// Block-wide maximum of a non-negative double, published with one unsigned
// 64-bit atomic max per block.  Every thread of the block must call it.
__device__ __forceinline__ void publish_max(unsigned long long *dst, double v)
{
    __shared__ double part[kBlock / kWave];
    v = wave_max(v);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = part[0];
#pragma unroll
        for (int w = 1; w < kBlock / kWave; ++w) m = fmax(m, part[w]);
        if (m > 0.0) atomicMax(dst, (unsigned long long)__double_as_longlong(m));
    }
}

// Block-wide maximum of a CFL ratio into the ratio word of this block's die.
__device__ __forceinline__ void publish_ratio(Slot &s, double v)
{
    publish_max(&s.r[blockIdx.x % kRatioWords].bits, v);
}

// Block-wide sum of a per-lane count, one atomic add per block if nonzero.
// Every thread of the block must call it.
__device__ __forceinline__ void publish_count(unsigned long long *dst, unsigned v)
{
    __shared__ unsigned part[kBlock / kWave];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
#pragma unroll
        for (int w = 0; w < kBlock / kWave; ++w) s += part[w];
        if (s) atomicAdd(dst, s);
    }
}

// record a non-physical value (h <= 0 or non-finite) produced by step `step`
__device__ __forceinline__ void flag_bad_at(const StepArgs &a, bool bad, long long step)
{
    if (bad) {
        atomicOr(&a.err->flag, 1u);
        atomicMin(&a.err->first_step, (unsigned long long)step);
    }
}

__device__ __forceinline__ void flag_bad(const StepArgs &a, bool bad)
{
    flag_bad_at(a, bad, a.slots[a.sa].step + 1);
}

template <int N>
__device__ __forceinline__ double lam_of(double g, double h, double ih, const double *q)
{
    double a[N + 1];
#pragma unroll
    for (int k = 0; k <= N; ++k) a[k] = q[k] * ih;
    return lam_bound<N>(g * h, a);
}

// CFL ratio r_i = sum_f |e_f| lam(Q_i, n_f) / (2 |V_i|) of one cell (the same
// expression in the step epilogue and in the stand-alone reduction, so a state
// reloaded from a checkpoint continues bitwise identically).
template <int N>
__device__ __forceinline__ double cfl_ratio_1d(double g, double h, double ih, const double *q, double idx,
                                               double *lmax)
{
    double l = lam_of<N>(g, h, ih, q);
    *lmax = l;
    return l * idx;
}

template <int N>
__device__ __forceinline__ double cfl_ratio_2d(double g, double h, double ih, const double *qx, const double *qy,
                                               double idx, double idy, double *lmax)
{
    double lx = lam_of<N>(g, h, ih, qx), ly = lam_of<N>(g, h, ih, qy);
    *lmax = fmax(lx, ly);
    return lx * idx + ly * idy;
}

// Unit normal and |e| / |V| of a triangle face from its scaled normal
// (sx, sy) = n |e| and the cell's 1 / |V|.  The two cells of a face hold
// exactly opposite scaled normals, so they derive exactly opposite unit
// normals.
__device__ __forceinline__ void face_geom(double sx, double sy, double ivol, double &nx, double &ny, double &w)
{
    const double el = sqrt_pos(fma(sx, sx, sy * sy));
    const double iel = rcp(el);
    nx = sx * iel;
    ny = sy * iel;
    w = el * ivol;
}

// geometry of the three faces of triangle i (internal order)
__device__ __forceinline__ void tri_geom(const StepArgs &a, int64_t i, double *nx, double *ny, double *w)
{
    const double iv = a.ivol[i];
#pragma unroll
    for (int s = 0; s < 3; ++s) face_geom(a.fsx[s * a.stride + i], a.fsy[s * a.stride + i], iv, nx[s], ny[s], w[s]);
}

template <int N>
__device__ __forceinline__ double cfl_ratio_tri(double g, double h, double ih, const double *qx, const double *qy,
                                                const double *fnx, const double *fny, const double *fw,
                                                double *lmax)
{
    const double gh = g * h;
    double r = 0.0, lm = 0.0;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        double an[N + 1];
#pragma unroll
        for (int k = 0; k <= N; ++k) an[k] = fma(qx[k], fnx[s], qy[k] * fny[s]) * ih;
        double l = lam_bound<N>(gh, an);
        lm = fmax(lm, l);
        r = fma(0.5 * fw[s], l, r);
    }
    *lmax = lm;
    return r;
}

// Cross-lane moves by one lane with DPP wave shifts (GFX9 wave_shl:1 /
// wave_shr:1): shfl_dn gives lane i the value of lane i + 1, shfl_up1 the
// value of lane i - 1; the lane without a source keeps its own value.
__device__ __forceinline__ double shfl_dn(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false),
                            __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double shfl_up1(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false),
                            __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false));
}

// Source column / row for a (possibly ghost) index along one axis.
// Returns the index to load and whether the normal momenta are mirrored.
__device__ __forceinline__ int ghost_index(int c, int n, int bc_lo, int bc_hi, bool &mirror)
{
    mirror = false;
    if (c < 0) {
        if (bc_lo == BC_PERIODIC) return n - 1;
        mirror = (bc_lo == BC_WALL);
        return 0;
    }
    if (c >= n) {
        if (c == n) {
            if (bc_hi == BC_PERIODIC) return 0;
            mirror = (bc_hi == BC_WALL);
        }
        return n - 1;
    }
    return c;
}

inline unsigned blocks_for(int64_t threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }

}  // namespace detail
}  // namespace sme

#define SME_LEVEL_SWITCH(level, CALL) \
    switch (level) {                  \
    case 0: CALL(0); break;           \
    case 1: CALL(1); break;           \
    case 2: CALL(2); break;           \
    case 3: CALL(3); break;           \
    case 4: CALL(4); break;           \
    case 5: CALL(5); break;           \
    case 6: CALL(6); break;           \
    case 7: CALL(7); break;           \
    case 8: CALL(8); break;           \
    default: return hipErrorInvalidValue; \
    }

