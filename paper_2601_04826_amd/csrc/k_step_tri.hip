// k_step_tri.hip -- SME step on triangle meshes (one launch per step).
#include <hip/hip_runtime.h>

#include "sme_step_common.h"

namespace sme {

using namespace detail;

namespace {

// ----------------------------------------------------------------------------
// Triangles: one lane per cell (internal order), faces s = 0, 1, 2.
template <int N>
__device__ __forceinline__ void frame_side(Side<N, true> &S, double h, double b, const double *qx, const double *qy,
                                           double nx, double ny, double g)
{
    S.h = h;
    S.b = b;
#pragma unroll
    for (int k = 0; k <= N; ++k) {
        S.qa[k] = fma(qx[k], nx, qy[k] * ny);
        S.qt[k] = fma(qy[k], nx, -qx[k] * ny);
    }
    side_flux<N, true>(S, g);
}

// Field access.  Up to level kTriBufLevel through buffer descriptors: each
// field is a uniform base (the descriptor, in scalar registers) and a lane's
// element a 32-bit byte offset, so a gather of all fields of one cell costs
// one offset, not one 64-bit address per field (nor the registers of those
// addresses: at level 3 the kernel fits three waves per SIMD instead of two).
// Triangle meshes hold at most 2^28 cells (checked when the mesh is read), so
// every offset fits in 32 bits.  Above that level the descriptors of the many
// fields no longer fit the scalar registers, and plain 64-bit addresses are
// used.  Measured per level at 1 M triangles: the buffer path is 2-7 % faster
// at levels 0-3 (three waves per SIMD at level 3); at level 4 (two waves per
// SIMD either way) 64-bit addresses with the next face's loads in flight are
// fastest; at levels 5-8 64-bit addresses without them (two waves per SIMD at
// levels 5-6 instead of one or two).
constexpr int kTriBufLevel = 3;
constexpr int kTriPrefetchLevel = 4;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const void *base, int64_t bytes)
{
    const unsigned nrec = bytes > 0xFFFFFFFFll ? 0xFFFFFFFFu : (unsigned)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)nrec, 0x00020000);
}

// element e of the field at base (stride elements per field)
template <bool BUF>
__device__ __forceinline__ double ld(const double *base, int64_t stride, int64_t e)
{
    if constexpr (BUF)
        return __builtin_bit_cast(double,
                                  __builtin_amdgcn_raw_buffer_load_b64(rsrc_of(base, stride * 8), (unsigned)e * 8u, 0, 0));
    else
        return base[e];
}

template <bool BUF>
__device__ __forceinline__ int ld_i32(const int32_t *base, int64_t stride, int64_t e)
{
    if constexpr (BUF)
        return (int)__builtin_amdgcn_raw_buffer_load_b32(rsrc_of(base, stride * 4), (unsigned)e * 4u, 0, 0);
    else
        return base[e];
}

template <bool BUF>
__device__ __forceinline__ void st(double v, double *base, int64_t stride, int64_t e)
{
    if constexpr (BUF)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v),
                                              rsrc_of(base, stride * 8), (unsigned)e * 8u, 0, 0);
    else
        base[e] = v;
}

// Raw state of one cell.
template <int N>
struct Raw {
    double h, b, qx[N + 1], qy[N + 1];
};

template <int N, bool BUF>
__device__ __forceinline__ void load_raw(const StepArgs &a, int64_t e, Raw<N> &r)
{
    constexpr int n = N + 1;
    r.h = ld<BUF>(a.q, a.stride, e);
    r.b = ld<BUF>(a.b, a.stride, e);
#pragma unroll
    for (int k = 0; k < n; ++k) {
        r.qx[k] = ld<BUF>(a.q + (1 + k) * a.stride, a.stride, e);
        r.qy[k] = ld<BUF>(a.q + (1 + n + k) * a.stride, a.stride, e);
    }
}

// What face s of cell i needs from memory besides its neighbour's index j (a
// wall if j < 0): the neighbour's raw state (the cell's own for a wall,
// mirrored at use) and the face's scaled normal n |e|.
template <int N>
struct FaceIn {
    int j;
    Raw<N> c;
    double sx, sy;
};

template <int N, bool BUF>
__device__ __forceinline__ void load_face(const StepArgs &a, int64_t i, int s, int j, FaceIn<N> &f)
{
    const int64_t so = s * a.stride;
    f.j = j;
    load_raw<N, BUF>(a, j < 0 ? i : j, f.c);
    f.sx = ld<BUF>(a.fsx + so, a.stride, i);
    f.sy = ld<BUF>(a.fsy + so, a.stride, i);
}

// IMP: the friction step is backward Euler (compile-time copy of the flag)
template <int N, bool IMP>
__global__ __launch_bounds__(kBlock) void k_step_tri(StepArgs a)
{
    constexpr int n = N + 1;
    constexpr int nf = 2 * n + 1;
    constexpr bool BUF = N <= kTriBufLevel;
    constexpr bool PRE = N == kTriPrefetchLevel;
    const double dt = step_dt(a);
    if (blockIdx.x == 0 && threadIdx.x == 0) slot_update(a, dt);
    if (dt == 0.0) {
        noop_step(a, nf);
        return;
    }
    // XCD-aware order: block b runs on die b % kXcd; each die gets one
    // contiguous range of the (bandwidth-reduced) cell order, so the neighbour
    // gathers of a die hit its own L2 instead of being fetched by every die
    const int64_t per_xcd = ((int64_t)gridDim.x + kXcd - 1) / kXcd;
    const int64_t slot = (int64_t)(blockIdx.x % kXcd) * per_xcd + blockIdx.x / kXcd;
    const int64_t i = slot * kBlock + threadIdx.x;
    double r = 0.0;
    if (i < a.ncells) {
        Raw<N> c0;
        load_raw<N, BUF>(a, i, c0);
        const double iv = ld<BUF>(a.ivol, a.stride, i);
        double acc[nf];
#pragma unroll
        for (int f = 0; f < nf; ++f) acc[f] = 0.0;
        // One face at a time (rolled: the live set is one face's two sides).
        // With PRE the loads of the next face are issued before the current
        // face is evaluated: their registers against their latency, which
        // pays where the kernel runs two waves per SIMD either way.
        FaceIn<N> nxt;
        int jn[3];
        if constexpr (PRE) {
#pragma unroll
            for (int s = 0; s < 3; ++s) jn[s] = ld_i32<BUF>(a.nbr + s * a.stride, a.stride, i);
            load_face<N, BUF>(a, i, 0, jn[0], nxt);
        }
#pragma unroll 1
        for (int s = 0; s < 3; ++s) {
            FaceIn<N> cur;
            if constexpr (PRE) {
                cur = nxt;
                if (s < 2) load_face<N, BUF>(a, i, s + 1, s == 0 ? jn[1] : jn[2], nxt);
            } else {
                load_face<N, BUF>(a, i, s, ld_i32<BUF>(a.nbr + s * a.stride, a.stride, i), cur);
            }
            const int j = cur.j;
            Raw<N> &c1 = cur.c;
            double nx, ny, w;
            face_geom(cur.sx, cur.sy, iv, nx, ny, w);
            if (j < 0) {  // reflective wall: mirror the normal momenta
                c1.h = c0.h;
                c1.b = c0.b;
#pragma unroll
                for (int k = 0; k < n; ++k) {
                    double qn = fma(c0.qx[k], nx, c0.qy[k] * ny);
                    c1.qx[k] = fma(-2.0 * qn, nx, c0.qx[k]);
                    c1.qy[k] = fma(-2.0 * qn, ny, c0.qy[k]);
                }
            }
            // canonical orientation: from the lower to the higher cell index,
            // so both cells of a face evaluate it on bitwise equal inputs
            const bool own_left = (j < 0) || (i < j);
            const double sx = own_left ? nx : -nx;
            const double sy = own_left ? ny : -ny;
            double qxl[n], qyl[n], qxr[n], qyr[n];
#pragma unroll
            for (int k = 0; k < n; ++k) {
                qxl[k] = own_left ? c0.qx[k] : c1.qx[k];
                qyl[k] = own_left ? c0.qy[k] : c1.qy[k];
                qxr[k] = own_left ? c1.qx[k] : c0.qx[k];
                qyr[k] = own_left ? c1.qy[k] : c0.qy[k];
            }
            Side<N, true> L, R;
            frame_side<N>(L, own_left ? c0.h : c1.h, own_left ? c0.b : c1.b, qxl, qyl, sx, sy, a.g);
            frame_side<N>(R, own_left ? c1.h : c0.h, own_left ? c1.b : c0.b, qxr, qyr, sx, sy, a.g);
            double Fh[nf], D[nf];
            face_flux<N, true>(L, R, a.g, a.quad, Fh, D);
            // this cell's share, rotated from the frame (a, t) with normal (sx, sy) back to (x, y)
            const double sgn = own_left ? 1.0 : -1.0;
            acc[0] = fma(w, fma(0.5, D[0], sgn * Fh[0]), acc[0]);
#pragma unroll
            for (int k = 0; k < n; ++k) {
                const double ca = fma(0.5, D[1 + k], sgn * Fh[1 + k]);
                const double ct = fma(0.5, D[1 + n + k], sgn * Fh[1 + n + k]);
                acc[1 + k] = fma(w, fma(ca, sx, -ct * sy), acc[1 + k]);
                acc[1 + n + k] = fma(w, fma(ca, sy, ct * sx), acc[1 + n + k]);
            }
        }
        double h = fma(-dt, acc[0], c0.h);
        double qx[n], qy[n];
#pragma unroll
        for (int k = 0; k < n; ++k) {
            qx[k] = fma(-dt, acc[1 + k], c0.qx[k]);
            qy[k] = fma(-dt, acc[1 + n + k], c0.qy[k]);
        }
        const double ih = rcp(h);
        friction_step<N, true, IMP>(qx, qy, ih, dt, a.c_slip, a.nu);
        st<BUF>(h, a.qn, a.stride, i);
        bool bad = !(h > 0.0) || !isfinite(h);
#pragma unroll
        for (int k = 0; k < n; ++k) {
            st<BUF>(qx[k], a.qn + (1 + k) * a.stride, a.stride, i);
            st<BUF>(qy[k], a.qn + (1 + n + k) * a.stride, a.stride, i);
            bad |= !isfinite(qx[k]) || !isfinite(qy[k]);
        }
        flag_bad(a, bad);
        // the face geometry again (cached) rather than held across the face loop
        double fw[3], fnx[3], fny[3];
#pragma unroll
        for (int s = 0; s < 3; ++s)
            face_geom(ld<BUF>(a.fsx + s * a.stride, a.stride, i), ld<BUF>(a.fsy + s * a.stride, a.stride, i), iv,
                      fnx[s], fny[s], fw[s]);
        double lm;
        r = cfl_ratio_tri<N>(a.g, h, ih, qx, qy, fnx, fny, fw, &lm);
        if (!(r >= 0.0)) r = 0.0;
    }
    publish_ratio(a.slots[a.sb], r);
}

}  // namespace

hipError_t launch_step_tri(int level, const StepArgs &a, hipStream_t s)
{
    // whole dies' worth of blocks, so the die-major slot order covers every cell
    const unsigned grid = (blocks_for(a.ncells) + kXcd - 1) / kXcd * kXcd;
#define L3(N) hipLaunchKernelGGL((k_step_tri<N, false>), dim3(grid), dim3(kBlock), 0, s, a)
#define L3X(N) hipLaunchKernelGGL((k_step_tri<N, true>), dim3(grid), dim3(kBlock), 0, s, a)
    if (a.implicit) {
        SME_LEVEL_SWITCH(level, L3X)
    } else {
        SME_LEVEL_SWITCH(level, L3)
    }
#undef L3
#undef L3X
    return hipGetLastError();
}

}  // namespace sme
