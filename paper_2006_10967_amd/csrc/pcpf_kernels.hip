// HIP kernels of the FR-PCPF residual for gfx950 (tensor-product quads/hexes).
//
// Work decomposition: one thread per solution point, EPB whole elements per block, the
// element data staged in LDS. Every element operator of the tensor-product element acts
// along one reference direction at a time (line form): the interpolation to a face point
// reads the p+1 points of one line, the derivative along xi_k reads the line through the
// point, and the correction (lifting) functions of a face touch only the line ending at
// that face point. This is the sum-factorised form of the dense operators of §3.1
// (Steps 1, 3, 4 and 6), exact in exact arithmetic.
//
// LDG orientation (§3.1 Step 2 with beta = +-1/2): the element on the - side of a face
// owns it. Its common solution is the neighbour's trace (so only + faces carry a jump in
// the corrected gradient), and it computes the common normal flux (Step 5) from its own
// viscous flux. Hence only two fields cross element boundaries per stage: the traces on
// - faces (read by the owner) and the common flux on + faces (read back by the neighbour
// with the opposite sign). Boundary faces (no neighbour) use the ghost state B(u) = u,
// B(q) = q of §3.3 and are computed by the element itself.
#include <cmath>

#include "pcpf_internal.h"

namespace pcpf {
namespace {

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
};
template <>
struct Math<float> {
    __device__ static float sqrt_(float x) { return ::sqrtf(x); }
    __device__ static void sincospi_(float x, float* s, float* c) { ::sincospif(x, s, c); }
    __device__ static float tanh_(float x) { return ::tanhf(x); }
    __device__ static float log10_(float x) { return ::log10f(x); }
    __device__ static float sinpi_(float x) { return ::sinpif(x); }
    __device__ static float fabs_(float x) { return ::fabsf(x); }
};

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
        v[0] = A * (R(0.5) - x[1]);
        v[1] = A * (x[0] - R(0.5));
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

template <typename R>
__device__ __forceinline__ R visc_ramp(R e_all, R e_top, R s0, R kappa, R nu_max) {
    // §3.2: s_e = log10(<u-u^,u-u^>/<u,u>), smooth ramp of half width kappa around s0
    if (!(e_all > R(0)) || !(e_top > R(0))) return R(0);
    const R s = Math<R>::log10_(e_top / e_all);
    if (s < s0 - kappa) return R(0);
    if (s > s0 + kappa) return nu_max;
    return R(0.5) * nu_max * (R(1) + Math<R>::sinpi_((s - s0) / (R(2) * kappa)));
}

// ------------------------------------------------------------------------------------
// grad_flux: Steps 1-5 for the elements of one block.
//   GF_PHYS     u = [phi, psi]: corrected gradients, fluxes at solution points, partial
//               divergence P = sum_k DH_k f~_k, common fluxes on owned faces.
//   GF_PRECOND  psi only: sensor nu_e, g = -nu_e grad psi, source S = sgn (1 - |q|),
//               P = sum_k DH_k g~_k - |J| S, common fluxes on owned faces.
//   GF_SIGN     psi0 only: smeared sign tanh(psi0 / max(|grad psi0|, delta_g)).
//   GF_SENSOR   psi only: the element viscosity nu_e.
// ------------------------------------------------------------------------------------
template <typename R, int D, int P, int MODE>
__global__ __launch_bounds__((Shape<D, P>::NT)) void k_grad_flux(GFArgs<R> a) {
    using S = Shape<D, P>;
    constexpr int N = S::N, NU = S::NU, NFA = S::NFA, EPB = S::EPB, NT = S::NT, G = S::GEO;
    constexpr int V = (MODE == GF_PHYS) ? 2 : 1;
    constexpr int NOPS = ops_size(N);
    constexpr bool FLUX = (MODE == GF_PHYS || MODE == GF_PRECOND);
    constexpr bool SENS = (MODE == GF_PRECOND || MODE == GF_SENSOR);
    constexpr bool GRAD = (MODE != GF_SENSOR);
    constexpr int NFE = 2 * D * NFA;     // face points per element
    using M = Math<R>;

    __shared__ R s_ops[NOPS];
    __shared__ R s_geo[EPB * G];
    __shared__ R s_u[V][EPB * NU];
    __shared__ R s_q[GRAD ? V : 1][D][GRAD ? EPB * NU : 1];
    __shared__ R s_f[FLUX ? V : 1][D][FLUX ? EPB * NU : 1];
    __shared__ R s_own[V][GRAD ? EPB * NFE : 1];
    __shared__ R s_nbr[V][GRAD ? EPB * NFE : 1];
    __shared__ R s_tmp[SENS ? 2 : 1][SENS ? EPB * NU : 1];
    __shared__ R s_nu[EPB];

    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    const int nel = (int)((a.E - e0) < EPB ? (a.E - e0) : EPB);

    for (int i = tid; i < NOPS; i += NT) s_ops[i] = a.ops[i];
    for (int i = tid; i < nel * G; i += NT) s_geo[i] = a.geo[e0 * G + i];
#pragma unroll
    for (int v = 0; v < V; ++v)
        for (int i = tid; i < nel * NU; i += NT) s_u[v][i] = a.u[v][e0 * NU + i];
    __syncthreads();

    const bool pt = tid < nel * NU;
    const int le = tid / NU;
    const int ip = tid - le * NU;
    int mi[D];
    {
        int r = ip;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            mi[k] = r % N;
            r /= N;
        }
    }

    // --- sensor (§3.2): modal coefficients by one 1D transform per direction ----------
    if constexpr (SENS) {
        const R* VI = &s_ops[op_vinv(N)];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const R* src = (k == 0) ? s_u[0] : s_tmp[(k - 1) & 1];
            R* dst = s_tmp[k & 1];
            if (pt) {
                R acc = R(0);
                const int b0 = le * NU + ip - mi[k] * st<N>(k);
#pragma unroll
                for (int q = 0; q < N; ++q) acc += VI[mi[k] * N + q] * src[b0 + q * st<N>(k)];
                dst[tid] = acc;
            }
            __syncthreads();
        }
        const R* chi = s_tmp[(D - 1) & 1];
        if (tid < nel) {
            R ea = R(0), et = R(0);
            for (int i = 0; i < NU; ++i) {
                const R c = chi[tid * NU + i];
                ea += c * c;
                int r = i, top = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    top |= ((r % N) == P);
                    r /= N;
                }
                if (top) et += c * c;
            }
            const R nu = visc_ramp(ea, et, a.ph.s0, a.ph.kappa, a.ph.nu_max);
            s_nu[tid] = nu;
            if constexpr (MODE == GF_SENSOR) a.out[e0 + tid] = nu;
        }
        __syncthreads();
        if constexpr (MODE == GF_SENSOR) return;
    }

    if constexpr (GRAD) {
        // --- Step 1 + 2: traces on owned faces and the neighbour's traces ------------------
        for (int it = tid; it < nel * NFE; it += NT) {
            const int el = it / NFE;
            const int r = it - el * NFE;
            const int f = r / NFA;
            const int t = r - f * NFA;
            const int k = f >> 1, s = f & 1;
            const int32_t en = a.nbr[(e0 + el) * 2 * D + f];
            if (s == 0 && en >= 0) continue;
            const int base = el * NU + face_base<D, N>(k, t);
            const R* l = &s_ops[s ? op_lp(N) : op_lm(N)];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R own = R(0);
#pragma unroll
                for (int q = 0; q < N; ++q) own += l[q] * s_u[v][base + q * st<N>(k)];
                const R nb = (en >= 0) ? a.Tm[v][((int64_t)en * D + k) * NFA + t] : own;
                s_own[v][it] = own;
                s_nbr[v][it] = nb;
            }
        }
        __syncthreads();

        // --- Step 3 (+ Step 4): corrected gradient and fluxes at solution points -----------
        R det = R(1);
        R Sdet = R(0);
        if (pt) {
            const R* gg = &s_geo[le * G];
            det = gg[D + 2 * D * D];
            const R* Ji = gg + D + D * D;        // Jinv[k][i] = Ji[k*D + i]
            const R* D1 = &s_ops[OP_D1];
            const R* cp = &s_ops[op_cp(N)];
            R q[V][D];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R qt[D];
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const int b0 = le * NU + ip - mi[k] * st<N>(k);
                    R acc = R(0);
#pragma unroll
                    for (int b = 0; b < N; ++b) acc += D1[mi[k] * N + b] * s_u[v][b0 + b * st<N>(k)];
                    const int jx = le * NFE + (2 * k + 1) * NFA + tang_index<D, N>(k, mi);
                    acc += cp[mi[k]] * (s_nbr[v][jx] - s_own[v][jx]);
                    qt[k] = acc;
                }
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    R acc = R(0);
#pragma unroll
                    for (int k = 0; k < D; ++k) acc += Ji[k * D + i] * qt[k];
                    q[v][i] = acc;
                    s_q[v][i][tid] = acc;
                }
            }
            if constexpr (MODE == GF_SIGN) {
                R g2 = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) g2 += q[0][i] * q[0][i];
                R g = M::sqrt_(g2);
                if (!(g > a.ph.delta_g)) g = a.ph.delta_g;
                a.out[(e0 + le) * NU + ip] = M::tanh_(s_u[0][tid] / g);
            }
            if constexpr (MODE == GF_PHYS) {
                const R* xi = &s_ops[op_xi(N)];
                R x[D], vel[D];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    R acc = gg[i];
#pragma unroll
                    for (int j = 0; j < D; ++j) acc += gg[D + i * D + j] * (xi[mi[j]] + R(1));
                    x[i] = acc;
                }
                velocity<R, D>(a.ph, x, vel);
                R v2 = R(0), g2 = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    v2 += vel[i] * vel[i];
                    g2 += q[1][i] * q[1][i];
                }
                R mm = M::sqrt_(v2);
                if (!(mm > a.ph.gamma)) mm = a.ph.gamma;
                const R rn = R(1) / M::sqrt_(g2 + a.ph.delta_n * a.ph.delta_n);
                const R phi = s_u[0][tid], psi = s_u[1][tid];
                const R sharp = a.ph.gamma * phi * (R(1) - phi) * rn;
                R f0[D], f1[D];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const R fvis = mm * (a.ph.eps * q[0][i] - sharp * q[1][i]);
                    f0[i] = phi * vel[i] - fvis;
                    f1[i] = psi * vel[i];
                }
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    R a0 = R(0), a1 = R(0);
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        a0 += Ji[k * D + i] * f0[i];
                        a1 += Ji[k * D + i] * f1[i];
                    }
                    s_f[0][k][tid] = det * a0;
                    s_f[V - 1][k][tid] = det * a1;
                }
            }
            if constexpr (MODE == GF_PRECOND) {
                const R nu = s_nu[le];
                R g2 = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) g2 += q[0][i] * q[0][i];
                Sdet = det * a.sgn[(e0 + le) * NU + ip] * (R(1) - M::sqrt_(g2));
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    R acc = R(0);
#pragma unroll
                    for (int i = 0; i < D; ++i) acc += Ji[k * D + i] * q[0][i];
                    s_f[0][k][tid] = -det * nu * acc;
                }
            }
        }
        if constexpr (MODE == GF_SIGN) return;
        __syncthreads();

        // --- Step 6 (volume part): P = sum_k DH_k f~_k (- |J| S) ------------------------
        if (pt) {
            const R* DH = &s_ops[op_dh(N)];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R acc = R(0);
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const int b0 = le * NU + ip - mi[k] * st<N>(k);
#pragma unroll
                    for (int b = 0; b < N; ++b) acc += DH[mi[k] * N + b] * s_f[v][k][b0 + b * st<N>(k)];
                }
                if constexpr (MODE == GF_PRECOND) acc -= Sdet;
                a.P[v][(e0 + le) * NU + ip] = acc;
            }
        }

        // --- Step 5: common normal fluxes on owned faces -----------------------------------
        for (int it = tid; it < nel * NFE; it += NT) {
            const int el = it / NFE;
            const int r = it - el * NFE;
            const int f = r / NFA;
            const int t = r - f * NFA;
            const int k = f >> 1, s = f & 1;
            const int64_t e = e0 + el;
            const int32_t en = a.nbr[e * 2 * D + f];
            if (s == 0 && en >= 0) continue;
            const int base = el * NU + face_base<D, N>(k, t);
            const R* l = &s_ops[s ? op_lp(N) : op_lm(N)];
            const R* gg = &s_geo[el * G];
            const R* Ji = gg + D + D * D;
            const R det_e = gg[D + 2 * D * D];
            R mag2 = R(0);
#pragma unroll
            for (int i = 0; i < D; ++i) mag2 += Ji[k * D + i] * Ji[k * D + i];
            const R mag = M::sqrt_(mag2);
            const R sgn_n = s ? R(1) : R(-1);
            R nrm[D];
#pragma unroll
            for (int i = 0; i < D; ++i) nrm[i] = sgn_n * Ji[k * D + i] / mag;
            const R sc = det_e * mag;
            R qn[V];      // own corrected gradient at the face point, dotted with n
            R qf1[D];     // psi gradient at the face point (normal of the sharpening term)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R acc_n = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    R acc = R(0);
#pragma unroll
                    for (int q = 0; q < N; ++q) acc += l[q] * s_q[v][i][base + q * st<N>(k)];
                    acc_n += acc * nrm[i];
                    if (v == V - 1) qf1[i] = acc;
                }
                qn[v] = acc_n;
            }
            const int64_t fo = (e * D + k) * NFA + t;
            if constexpr (MODE == GF_PHYS) {
                const R* xi = &s_ops[op_xi(N)];
                R xr[D];
                {
                    int tt = t;
#pragma unroll
                    for (int m = 0; m < D; ++m) {
                        if (m == k) {
                            xr[m] = s ? R(2) : R(0);
                        } else {
                            xr[m] = xi[tt % N] + R(1);
                            tt /= N;
                        }
                    }
                }
                R x[D], vel[D];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    R acc = gg[i];
#pragma unroll
                    for (int j = 0; j < D; ++j) acc += gg[D + i * D + j] * xr[j];
                    x[i] = acc;
                }
                velocity<R, D>(a.ph, x, vel);
                R v2 = R(0), vn = R(0), g2 = R(0), gn = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    v2 += vel[i] * vel[i];
                    vn += vel[i] * nrm[i];
                    g2 += qf1[i] * qf1[i];
                }
                gn = qn[1];
                R mm = M::sqrt_(v2);
                if (!(mm > a.ph.gamma)) mm = a.ph.gamma;
                const R pL = s_own[0][it], pR = s_nbr[0][it];
                const R sL = s_own[1][it], sR = s_nbr[1][it];
                const R rn = R(1) / M::sqrt_(g2 + a.ph.delta_n * a.ph.delta_n);
                const R fvn = mm * (a.ph.eps * qn[0] - a.ph.gamma * pL * (R(1) - pL) * gn * rn);
                const R F0 = R(0.5) * (pL + pR) * vn - fvn + a.ph.tau * (pL - pR);
                const R F1 = R(0.5) * (sL + sR) * vn + a.ph.tau * (sL - sR);
                (s ? a.Fp[0] : a.Fbm[0])[fo] = sc * F0;
                (s ? a.Fp[1] : a.Fbm[1])[fo] = sc * F1;
            } else {
                const R sL = s_own[0][it], sR = s_nbr[0][it];
                const R F = -s_nu[el] * qn[0] + a.ph.tau * (sL - sR);
                (s ? a.Fp[0] : a.Fbm[0])[fo] = sc * F;
            }
        }
    }
}

// ------------------------------------------------------------------------------------
// update: Step 6 face part and the RK4 stage combine.
//   R = -(P + sum_faces c_face F~) / |J|; then either the residual is written (UP_RESID)
//   or the classic RK4 registers are advanced and the - face traces of the next stage
//   input are written (UP_RK).
// ------------------------------------------------------------------------------------
template <typename R, int D, int P, int V, int KIND>
__global__ __launch_bounds__((Shape<D, P>::NT)) void k_update(UPArgs<R> a) {
    using S = Shape<D, P>;
    constexpr int N = S::N, NU = S::NU, NFA = S::NFA, EPB = S::EPB, NT = S::NT, G = S::GEO;
    constexpr int NOPS = ops_size(N);
    constexpr int NFE = 2 * D * NFA;
    __shared__ R s_ops[NOPS];
    __shared__ R s_F[V][EPB * NFE];
    __shared__ R s_u[V][KIND == UP_RK ? EPB * NU : 1];
    __shared__ R s_det[EPB];

    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    const int nel = (int)((a.E - e0) < EPB ? (a.E - e0) : EPB);
    for (int i = tid; i < NOPS; i += NT) s_ops[i] = a.ops[i];
    if (tid < nel) s_det[tid] = a.geo[(e0 + tid) * G + D + 2 * D * D];
    for (int it = tid; it < nel * NFE; it += NT) {
        const int el = it / NFE;
        const int r = it - el * NFE;
        const int f = r / NFA;
        const int t = r - f * NFA;
        const int k = f >> 1, s = f & 1;
        const int64_t e = e0 + el;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            R F;
            if (s) {
                F = a.Fp[v][(e * D + k) * NFA + t];
            } else {
                const int32_t en = a.nbr[e * 2 * D + f];
                F = (en >= 0) ? -a.Fp[v][((int64_t)en * D + k) * NFA + t]
                              : a.Fbm[v][(e * D + k) * NFA + t];
            }
            s_F[v][it] = F;
        }
    }
    __syncthreads();

    const bool pt = tid < nel * NU;
    if (pt) {
        const int le = tid / NU;
        const int ip = tid - le * NU;
        int mi[D];
        {
            int r = ip;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                mi[k] = r % N;
                r /= N;
            }
        }
        const R* cm = &s_ops[op_cm(N)];
        const R* cp = &s_ops[op_cp(N)];
        const int64_t idx = (e0 + le) * NU + ip;
        const R rdet = R(1) / s_det[le];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            R acc = a.P[v][idx];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int tk = tang_index<D, N>(k, mi);
                acc += cp[mi[k]] * s_F[v][le * NFE + (2 * k + 1) * NFA + tk]
                     + cm[mi[k]] * s_F[v][le * NFE + (2 * k) * NFA + tk];
            }
            const R res = -acc * rdet;
            if constexpr (KIND == UP_RESID) {
                a.res[v][idx] = res;
            } else {
                const R un = a.un[v][idx];
                R nx;
                if (!a.last) {
                    const R ac = (a.first ? R(0) : a.acc[v][idx]) + a.bcoef * res;
                    a.acc[v][idx] = ac;
                    nx = un + a.ccoef * res;
                    a.us[v][idx] = nx;
                } else {
                    nx = un + a.ccoef * (a.acc[v][idx] + a.bcoef * res);
                    a.un[v][idx] = nx;
                }
                s_u[v][tid] = nx;
                const R lim = (v == 0 && V == 2) ? R(10) : R(1e30);
                if (!(Math<R>::fabs_(nx) <= lim)) *a.flag = 1;
            }
        }
    }
    if constexpr (KIND == UP_RK) {
        __syncthreads();
        const R* lm = &s_ops[op_lm(N)];
        constexpr int NMF = D * NFA;
        for (int it = tid; it < nel * NMF; it += NT) {
            const int el = it / NMF;
            const int r = it - el * NMF;
            const int k = r / NFA;
            const int t = r - k * NFA;
            const int base = el * NU + face_base<D, N>(k, t);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R acc = R(0);
#pragma unroll
                for (int q = 0; q < N; ++q) acc += lm[q] * s_u[v][base + q * st<N>(k)];
                a.Tm[v][((e0 + el) * D + k) * NFA + t] = acc;
            }
        }
    }
}

// traces on - faces of a given state (after set_state / reset)
template <typename R, int D, int P, int V>
__global__ __launch_bounds__((Shape<D, P>::NT)) void k_trace(TRArgs<R> a) {
    using S = Shape<D, P>;
    constexpr int N = S::N, NU = S::NU, NFA = S::NFA, EPB = S::EPB, NT = S::NT;
    __shared__ R s_lm[N];
    __shared__ R s_u[V][EPB * NU];
    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    const int nel = (int)((a.E - e0) < EPB ? (a.E - e0) : EPB);
    if (tid < N) s_lm[tid] = a.ops[op_lm(N) + tid];
#pragma unroll
    for (int v = 0; v < V; ++v)
        for (int i = tid; i < nel * NU; i += NT) s_u[v][i] = a.u[v][e0 * NU + i];
    __syncthreads();
    constexpr int NMF = D * NFA;
    for (int it = tid; it < nel * NMF; it += NT) {
        const int el = it / NMF;
        const int r = it - el * NMF;
        const int k = r / NFA;
        const int t = r - k * NFA;
        const int base = el * NU + face_base<D, N>(k, t);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            R acc = R(0);
#pragma unroll
            for (int q = 0; q < N; ++q) acc += s_lm[q] * s_u[v][base + q * st<N>(k)];
            a.Tm[v][((e0 + el) * D + k) * NFA + t] = acc;
        }
    }
}

// FP64 quadrature reduction, first pass: block partial sums in a fixed order.
__device__ __forceinline__ double block_sum(double x) {
    __shared__ double s_w[REDUCE_THREADS / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s_w[w] = x;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < REDUCE_THREADS / 64; ++i) r += s_w[i];
    }
    return r;
}

template <typename R, int D, int P>
__global__ __launch_bounds__(REDUCE_THREADS) void k_reduce(RDArgs<R> a) {
    using S = Shape<D, P>;
    constexpr int N = S::N, NU = S::NU;
    const int64_t total = a.E * NU;
    double acc = 0.0;
    for (int64_t idx = (int64_t)blockIdx.x * REDUCE_THREADS + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * REDUCE_THREADS) {
        const int64_t e = idx / NU;
        int r = (int)(idx - e * NU);
        double W = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            W *= a.w64[r % N];
            r /= N;
        }
        double f = (double)a.field[idx];
        if (a.kind == 1) f = ::fabs(f - (double)a.ref[idx]);
        acc += a.det64[e] * W * f;
    }
    const double b = block_sum(acc);
    if (threadIdx.x == 0) a.partial[blockIdx.x] = b;
}

__global__ __launch_bounds__(REDUCE_THREADS) void k_reduce_final(const double* partial, int nb,
                                                                double* out) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += REDUCE_THREADS) acc += partial[i];
    const double b = block_sum(acc);
    if (threadIdx.x == 0) *out = b;
}

template <typename R>
__global__ void k_reset(const R* phi, R* psi, int64_t n, int mode, double eps_w, double dphi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (mode == PCPF_RESET_LOGIT) {
        double c = (double)phi[i];
        c = c < dphi ? dphi : (c > 1.0 - dphi ? 1.0 - dphi : c);
        psi[i] = (R)(eps_w * ::log(c / (1.0 - c)));
    } else {
        psi[i] = phi[i] - R(0.5);
    }
}

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------
template <typename R, int D, int P>
struct Impl {
    using S = Shape<D, P>;
    static unsigned grid(int64_t E) { return (unsigned)((E + S::EPB - 1) / S::EPB); }

    static void grad_flux(int mode, int nvar, const GFArgs<R>& a, hipStream_t st) {
        (void)nvar;
        const dim3 g(grid(a.E)), b(S::NT);
        switch (mode) {
            case GF_PHYS: hipLaunchKernelGGL((k_grad_flux<R, D, P, GF_PHYS>), g, b, 0, st, a); break;
            case GF_PRECOND: hipLaunchKernelGGL((k_grad_flux<R, D, P, GF_PRECOND>), g, b, 0, st, a); break;
            case GF_SIGN: hipLaunchKernelGGL((k_grad_flux<R, D, P, GF_SIGN>), g, b, 0, st, a); break;
            default: hipLaunchKernelGGL((k_grad_flux<R, D, P, GF_SENSOR>), g, b, 0, st, a); break;
        }
    }
    static void update(int kind, int nvar, const UPArgs<R>& a, hipStream_t st) {
        const dim3 g(grid(a.E)), b(S::NT);
        if (nvar == 2) {
            if (kind == UP_RK) hipLaunchKernelGGL((k_update<R, D, P, 2, UP_RK>), g, b, 0, st, a);
            else hipLaunchKernelGGL((k_update<R, D, P, 2, UP_RESID>), g, b, 0, st, a);
        } else {
            if (kind == UP_RK) hipLaunchKernelGGL((k_update<R, D, P, 1, UP_RK>), g, b, 0, st, a);
            else hipLaunchKernelGGL((k_update<R, D, P, 1, UP_RESID>), g, b, 0, st, a);
        }
    }
    static void trace(int nvar, const TRArgs<R>& a, hipStream_t st) {
        const dim3 g(grid(a.E)), b(S::NT);
        if (nvar == 2) hipLaunchKernelGGL((k_trace<R, D, P, 2>), g, b, 0, st, a);
        else hipLaunchKernelGGL((k_trace<R, D, P, 1>), g, b, 0, st, a);
    }
};

template <typename R, int D, int P>
void reduce_launch(const RDArgs<R>& a, int nblocks, hipStream_t st);

template <typename R, int D, int P>
bool fill(Launchers<R>* L) {
    using S = Shape<D, P>;
    L->epb = S::EPB;
    L->nt = S::NT;
    L->ngeo = S::GEO;
    L->grad_flux = &Impl<R, D, P>::grad_flux;
    L->update = &Impl<R, D, P>::update;
    L->trace = &Impl<R, D, P>::trace;
    L->reduce = &reduce_launch<R, D, P>;
    return true;
}

}  // namespace

namespace {
template <typename R, int D, int P>
void reduce_launch(const RDArgs<R>& a, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL((k_reduce<R, D, P>), dim3(nblocks), dim3(REDUCE_THREADS), 0, st, a);
}
}  // namespace

template <typename R>
bool get_launchers(int d, int p, Launchers<R>* L) {
    if (d == 2) {
        switch (p) {
            case 1: return fill<R, 2, 1>(L);
            case 2: return fill<R, 2, 2>(L);
            case 3: return fill<R, 2, 3>(L);
            case 4: return fill<R, 2, 4>(L);
            case 5: return fill<R, 2, 5>(L);
            case 6: return fill<R, 2, 6>(L);
            default: return false;
        }
    }
    if (d == 3) {
        switch (p) {
            case 1: return fill<R, 3, 1>(L);
            case 2: return fill<R, 3, 2>(L);
            case 3: return fill<R, 3, 3>(L);
            case 4: return fill<R, 3, 4>(L);
            case 5: return fill<R, 3, 5>(L);
            default: return false;
        }
    }
    return false;
}

template bool get_launchers<double>(int, int, Launchers<double>*);
template bool get_launchers<float>(int, int, Launchers<float>*);

template <typename R>
void launch_reset(const R* phi, R* psi, int64_t n, int mode, double eps_w, double delta_phi,
                  hipStream_t s) {
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL((k_reset<R>), dim3(g), dim3(256), 0, s, phi, psi, n, mode, eps_w, delta_phi);
}
template void launch_reset<double>(const double*, double*, int64_t, int, double, double, hipStream_t);
template void launch_reset<float>(const float*, float*, int64_t, int, double, double, hipStream_t);

void launch_reduce_final(const double* partial, int nblocks, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(REDUCE_THREADS), 0, s, partial, nblocks, out);
}

}  // namespace pcpf
