// Device helpers shared by the forward and adjoint kernels (tensor-product line indexing,
// analytic velocity fields, the viscosity ramp).
#pragma once

#include "pcpf_internal.h"

namespace pcpf {
namespace dev {

template <typename R>
struct Math;
template <>
struct Math<double> {
    __device__ static double sqrt_(double x) { return ::sqrt(x); }
    __device__ static void sincospi_(double x, double* s, double* c) { ::sincospi(x, s, c); }
    __device__ static double tanh_(double x) { return ::tanh(x); }
    __device__ static double log10_(double x) { return ::log10(x); }
    __device__ static double sinpi_(double x) { return ::sinpi(x); }
    __device__ static double fabs_(double x) { return ::fabs(x); }
    __device__ static double rsqrt_(double x) { return ::rsqrt(x); }
    __device__ static double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
};
template <>
struct Math<float> {
    __device__ static float sqrt_(float x) { return ::sqrtf(x); }
    __device__ static void sincospi_(float x, float* s, float* c) { ::sincospif(x, s, c); }
    __device__ static float tanh_(float x) { return ::tanhf(x); }
    __device__ static float log10_(float x) { return ::log10f(x); }
    __device__ static float sinpi_(float x) { return ::sinpif(x); }
    __device__ static float fabs_(float x) { return ::fabsf(x); }
    __device__ static float rsqrt_(float x) { return ::rsqrtf(x); }
    __device__ static float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
};

// Global accesses: a wave-uniform base pointer plus an unsigned 32-bit byte offset per
// lane (every array of a context is below 4 GiB, which pcpf_create checks). This selects
// the scalar-base + 32-bit-offset addressing of global loads and stores, which needs no
// 64-bit address arithmetic per lane.
template <typename T>
__device__ __forceinline__ T gld(const T* base, uint32_t i) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(T));
}
// Load of element min(i, n - 1) (n >= 1): an unconditional load that stays inside the n
// valid elements, for lanes whose value is then discarded. Without a branch around each
// load, the scalar loads of all base pointers can be issued together ahead of the vector
// loads instead of one after another.
template <typename T>
__device__ __forceinline__ T gld_in(const T* base, int i, int n) {
    return gld(base, (uint32_t)(i < n ? i : n - 1));
}
template <typename T>
__device__ __forceinline__ void gst(T* base, uint32_t i, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (uint32_t)sizeof(T)) = v;
}
// The same with the non-temporal hint (NT = true): for arrays a launch reads or writes once
// and that are too large to be found in the caches by the next launch.
template <bool NT, typename T>
__device__ __forceinline__ T gld_s(const T* base, uint32_t i) {
    const T* p = reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(T));
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void gst_s(T* base, uint32_t i, T v) {
    T* p = reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (uint32_t)sizeof(T));
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Element chunk of this block. Consecutive workgroups are placed round-robin on the 8
// XCDs. When a state plane is small enough for the chunks of one XCD to stay in its L2 and
// the shared cache between launches (at most 24 MiB; measured on the 2D and 3D meshes
// from 65 k to 7 M points), the chunks are renumbered so that each XCD takes one
// contiguous range: the faces its elements share (traces and fluxes pushed between
// neighbours) and the registers one launch writes and the next reads then stay with that
// XCD. Larger planes keep the concurrent blocks sweeping one address window, in runs of
// XCD_RUN consecutive chunks per XCD (rounds of 8 XCD_RUN blocks; a last partial round in
// plain order): the cache lines two consecutive chunks share are then fetched into one
// XCD's L2, not two (96^3 p4: stage 4059 -> 3925 us FP64, 2243 -> 2171 us FP32; the same
// within 1% from runs of 16 to 64). Either way a permutation: every chunk is processed
// exactly once.
constexpr int64_t XCD_MAP_MAX_PLANE_BYTES = int64_t(24) << 20;
constexpr uint32_t XCD_RUN = 32;

template <typename R>
__device__ __forceinline__ uint32_t block_chunk(int64_t points_per_plane) {
    const uint32_t b = blockIdx.x;
    constexpr uint32_t X = 8;
    const uint32_t g = gridDim.x;
    if (points_per_plane * (int64_t)sizeof(R) > XCD_MAP_MAX_PLANE_BYTES) {
        const uint32_t round = b / (X * XCD_RUN);
        if ((round + 1) * X * XCD_RUN > g) return b;
        return round * X * XCD_RUN + (b % X) * XCD_RUN + (b / X) % XCD_RUN;
    }
    const uint32_t x = b % X, q = g / X, r = g % X;
    return x * q + (x < r ? x : r) + b / X;
}

template <int N>
__device__ __forceinline__ constexpr int st(int k) {
    return k == 0 ? 1 : (k == 1 ? N : N * N);
}

// Solution-point index of the point at line position 0 of the line through face point t
// of a face normal to direction k (tangential indices ascending, first fastest).
template <int D, int N>
__device__ __forceinline__ int face_base(int k, int t) {
    int idx = 0;
#pragma unroll
    for (int m = 0; m < D; ++m) {
        if (m == k) continue;
        idx += (t % N) * st<N>(m);
        t /= N;
    }
    return idx;
}

// Face-point index, on the faces normal to k, of the line through point multi-index m.
template <int D, int N>
__device__ __forceinline__ int tang_index(int k, const int (&mi)[D]) {
    int t = 0, mul = 1;
#pragma unroll
    for (int q = 0; q < D; ++q) {
        if (q == k) continue;
        t += mi[q] * mul;
        mul *= N;
    }
    return t;
}

// v(x, t) = A g(t) v0(x) for the analytic fields of §4 (ampg = A g(t)).
template <typename R, int D>
__device__ __forceinline__ void velocity(const Phys<R>& ph, const R (&x)[D], R (&v)[D]) {
    using M = Math<R>;
    const R A = ph.ampg;
    if (ph.vel_kind == PCPF_VEL_UNIFORM) {
#pragma unroll
        for (int k = 0; k < D; ++k) v[k] = A * ph.u0[k];
    } else if (ph.vel_kind == PCPF_VEL_ROTATION) {
        v[0] = A * (ph.u0[1] - x[1]);      // rigid rotation about (u0[0], u0[1])
        v[1] = A * (x[0] - ph.u0[0]);
#pragma unroll
        for (int k = 2; k < D; ++k) v[k] = R(0);
    } else if (ph.vel_kind == PCPF_VEL_SINGLE_VORTEX) {
        R sx, cx, sy, cy;
        M::sincospi_(x[0], &sx, &cx);
        M::sincospi_(x[1], &sy, &cy);
        v[0] = A * (-(sx * sx) * (R(2) * sy * cy));
        v[1] = A * ((R(2) * sx * cx) * (sy * sy));
#pragma unroll
        for (int k = 2; k < D; ++k) v[k] = R(0);
    } else {
        R s[3], c[3];
#pragma unroll
        for (int k = 0; k < D; ++k) M::sincospi_(x[k], &s[k], &c[k]);
        if (D == 3) {
            const R s2x = R(2) * s[0] * c[0], s2y = R(2) * s[1] * c[1], s2z = R(2) * s[2] * c[2];
            v[0] = A * (R(2) * (s[0] * s[0]) * s2y * s2z);
            v[1] = A * (-s2x * (s[1] * s[1]) * s2z);
            v[D - 1] = A * (-s2x * s2y * (s[2] * s[2]));
        } else {
#pragma unroll
            for (int k = 0; k < D; ++k) v[k] = R(0);
        }
    }
}

// v(x, t) for the fields without trigonometric factors (uniform, rotation).
template <typename R, int D>
__device__ __forceinline__ void velocity_lin(const Phys<R>& ph, const R (&x)[D], R (&v)[D]) {
    const R A = ph.ampg;
    if (ph.vel_kind == PCPF_VEL_ROTATION) {
        v[0] = A * (ph.u0[1] - x[1]);      // rigid rotation about (u0[0], u0[1])
        v[1] = A * (x[0] - ph.u0[0]);
#pragma unroll
        for (int k = 2; k < D; ++k) v[k] = R(0);
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) v[k] = A * ph.u0[k];
    }
}

// max(sqrt(x), g) for x >= 0 and g > 0: the flux multiplier max(gamma, |v|) of §2. The root is
// taken only where x > g^2, which keeps its argument away from the tiny and huge ranges a
// general square root has to rescale. There the hardware reciprocal-root estimate y is
// refined by one step of Goldschmidt's coupled iteration for the pair
// (s, h) ~ (sqrt(x), 1/(2 sqrt(x))), started from (x y, y / 2): r = 1/2 - s h,
// s += s r, h += h r (quadratic convergence), then one Newton correction by the residual,
// s + h (x - s^2). With an estimate of relative error up to 2^-20 the result is within one
// ulp of the correctly rounded root (checked by exact emulation of every fused
// multiply-add on the CPU). NaN gives g, as max(sqrt(NaN), g) does.
__device__ __forceinline__ double max_sqrt(double x, double g) {
    if (!(x > g * g)) return g;
    const double y = __builtin_amdgcn_rsq(x);
    double s = x * y, h = 0.5 * y;
    const double r = __builtin_fma(-s, h, 0.5);
    s = __builtin_fma(s, r, s);
    h = __builtin_fma(h, r, h);
    const double d = __builtin_fma(-s, s, x);
    return __builtin_fma(d, h, s);
}
__device__ __forceinline__ float max_sqrt(float x, float g) {
    return (x > g * g) ? __builtin_amdgcn_sqrtf(x) : g;
}

template <typename R>
__device__ __forceinline__ R visc_ramp(R e_all, R e_top, R s0, R kappa, R nu_max) {
    // §3.2: s_e = log10(<u-u^,u-u^>/<u,u>), smooth ramp of half width kappa around s0
    if (!(e_all > R(0)) || !(e_top > R(0))) return R(0);
    const R s = Math<R>::log10_(e_top / e_all);
    if (s < s0 - kappa) return R(0);
    if (s > s0 + kappa) return nu_max;
    return R(0.5) * nu_max * (R(1) + Math<R>::sinpi_((s - s0) / (R(2) * kappa)));
}

// Velocity from the per-element tables of an axis-aligned element:
// vt[(k * NTB + pos_k) * 2 + {0, 1}] = (sin^2(pi x_k), sin(2 pi x_k)), pos_k the node index
// along k, or N / N + 1 for the xi_k = -1 / +1 end of the element.
template <typename R, int D, int NTB>
__device__ __forceinline__ void velocity_tab(const Phys<R>& ph, const R* vt, const int (&pos)[D],
                                             R (&v)[D]) {
    const R A = ph.ampg;
    R q[3], t[3];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        q[k] = vt[(k * NTB + pos[k]) * 2];
        t[k] = vt[(k * NTB + pos[k]) * 2 + 1];
    }
    if (ph.vel_kind == PCPF_VEL_SINGLE_VORTEX) {
        v[0] = A * (-q[0] * t[1]);
        v[1] = A * (t[0] * q[1]);
#pragma unroll
        for (int k = 2; k < D; ++k) v[k] = R(0);
    } else {
        if (D == 3) {
            v[0] = A * (R(2) * q[0] * t[1] * t[2]);
            v[1] = A * (-t[0] * q[1] * t[2]);
            v[D - 1] = A * (-t[0] * t[1] * q[2]);
        } else {
#pragma unroll
            for (int k = 0; k < D; ++k) v[k] = R(0);
        }
    }
}

}  // namespace dev
}  // namespace pcpf
