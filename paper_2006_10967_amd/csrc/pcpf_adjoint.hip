// Adjoint (reverse-mode) kernels of the FR-PCPF residuals for gfx950.
//
// For a stage input Y and the adjoint R^ of its residual R(Y) these kernels compute the
// vector-Jacobian product Y^ = (dR/dY)^T R^ (and dR/dA^T R^ for the velocity amplitude
// A) of the discrete operators the forward kernels apply: the line-form interpolation,
// corrected gradient and divergence operators are applied transposed, the pointwise and
// face fluxes are differentiated by hand, and every exchange between elements runs the
// other way round. The forward quantities of the stage (gradients, fluxes) are recomputed
// from Y, never stored.
//
// Per stage: k_adj_push (lifting adjoint of every - face and the forward trace of Y on it,
// both pushed to the owner of the face) -> k_adj_main (forward recompute + VJPs; trace
// adjoints pushed to the neighbours' - face slots) -> k_adj_finish (adds the pushed trace
// adjoints and performs the reverse RK4 combine).
#include <cmath>

#include "pcpf_adjoint.h"
#include "pcpf_device.h"

namespace pcpf {
namespace {

using namespace dev;

// ------------------------------------------------------------------------------------
// Push of one stage: F~^ of the - faces. The residual of element e contains
// cm * F~_slot / |J| with F~_slot = -F~_owner on faces that have an owner, so the owner's
// flux receives sum_a cm[a] R^(line a) / |J_e|. The same face points also carry the forward
// trace sum_a lm[a] Y(line a) that the owner's gradient reads (what the forward update
// pushes), so it is pushed here as well, in the same order of summation. Shared by
// k_adj_push and the tail of k_adj_finish: s_r / s_y hold R^ and Y of the block's elements.
// ------------------------------------------------------------------------------------
template <typename R, int D, int P, int V>
__device__ __forceinline__ void owners_of_minus_faces(int32_t* r_own, const int32_t* nbr, int64_t e0,
                                                      int nel, int tid) {
    using S = AShape<D, P>;
    constexpr int NMF = D * S::NFA;
    constexpr int I_T = (S::EPB * NMF + S::NT - 1) / S::NT;
#pragma unroll
    for (int j = 0; j < I_T; ++j) {
        const int it = tid + j * S::NT;
        const int el = it / NMF, k = (it - el * NMF) / S::NFA;
        r_own[j] = (it < nel * NMF) ? nbr[(e0 + el) * 2 * D + 2 * k] : -1;
    }
}

template <typename R, int D, int P, int V>
__device__ __forceinline__ void push_minus_faces(const R* s_cm, const R* s_lm, const R* const* s_r,
                                                 const R* const* s_y, const R* s_det,
                                                 const int32_t* r_own, R* const* gp, R* const* Tp,
                                                 int nel, int tid, int64_t E) {
    using S = AShape<D, P>;
    constexpr int N = S::N, NU = S::NU, NFA = S::NFA;
    constexpr int NMF = D * NFA;
    constexpr int I_T = (S::EPB * NMF + S::NT - 1) / S::NT;
#pragma unroll
    for (int j = 0; j < I_T; ++j) {
        const int it = tid + j * S::NT;
        if (it >= nel * NMF || r_own[j] < 0) continue;
        const int el = it / NMF, r = it - el * NMF, k = r / NFA, t = r - k * NFA;
        const int base = el * NU + face_base<D, N>(k, t);
        const R rd = R(1) / s_det[el];
        using M = Math<R>;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            R acc = R(0), tr = R(0);
#pragma unroll
            for (int q = 0; q < N; ++q) {
                acc = M::fma_(s_cm[q], s_r[v][base + q * st<N>(k)], acc);
                tr = M::fma_(s_lm[q], s_y[v][base + q * st<N>(k)], tr);
            }
            gp[v][((int64_t)r_own[j] * D + k) * NFA + t] = acc * rd;
            Tp[v][((int64_t)k * E + r_own[j]) * NFA + t] = tr;   // planar [D][E][NFA]
        }
    }
}

template <typename R, int D, int P, int V>
__global__ __launch_bounds__((AShape<D, P>::NT)) void k_adj_push(AJPush<R> a) {
    using S = AShape<D, P>;
    constexpr int N = S::N, NU = S::NU, NFA = S::NFA, EPB = S::EPB, NT = S::NT, G = S::GEO;
    constexpr int I_T = (EPB * D * NFA + NT - 1) / NT;
    constexpr int I_U = (EPB * NU + NT - 1) / NT;
    __shared__ R s_cm[N];
    __shared__ R s_lm[N];
    __shared__ R s_r[V][EPB * NU];
    __shared__ R s_y[V][EPB * NU];
    __shared__ R s_det[EPB];
    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    const int nel = (int)((a.E - e0) < EPB ? (a.E - e0) : EPB);
    int32_t r_own[I_T];
    owners_of_minus_faces<R, D, P, V>(r_own, a.nbr, e0, nel, tid);
    const bool seed = a.seed_yb[0] != nullptr;
    R r_r[V][I_U], r_y[V][I_U];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
        for (int j = 0; j < I_U; ++j) {
            const int i = tid + j * NT;
            if (seed) {
                r_r[v][j] = (i < nel * NU) ? a.seed_yb[v][e0 * NU + i] : R(0);
            } else {
                r_r[v][j] = (i < nel * NU) ? a.rbar[v][e0 * NU + i] : R(0);
            }
            r_y[v][j] = (i < nel * NU) ? a.u[v][e0 * NU + i] : R(0);
        }
    if (seed) {
        // ya <- yb, R^ = alpha yb + 0 (as the axpby of the plain sweep)
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int j = 0; j < I_U; ++j) {
                const int i = tid + j * NT;
                if (i < nel * NU) {
                    a.seed_ya[v][e0 * NU + i] = r_r[v][j];
                    r_r[v][j] = a.seed_alpha * r_r[v][j] + R(0);
                    a.seed_rb[v][e0 * NU + i] = r_r[v][j];
                }
            }
    }
    const R r_c = (tid < N) ? a.ops[op_cm(N) + tid] : R(0);
    const R r_l = (tid < N) ? a.ops[op_lm(N) + tid] : R(0);
    const R r_d = (tid < nel) ? a.geo[(e0 + tid) * G + D + 2 * D * D] : R(1);
    if (tid < N) {
        s_cm[tid] = r_c;
        s_lm[tid] = r_l;
    }
    if (tid < nel) s_det[tid] = r_d;
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
        for (int j = 0; j < I_U; ++j)
            if (tid + j * NT < nel * NU) {
                s_r[v][tid + j * NT] = r_r[v][j];
                s_y[v][tid + j * NT] = r_y[v][j];
            }
    __syncthreads();
    const R* sr[V];
    const R* sy[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        sr[v] = s_r[v];
        sy[v] = s_y[v];
    }
    push_minus_faces<R, D, P, V>(s_cm, s_lm, sr, sy, s_det, r_own, a.gp, a.Tp, nel, tid, a.E);
}

// ------------------------------------------------------------------------------------
// k_adj_main: forward recompute of one stage and the vector-Jacobian product.
//   AD_PHYS     u = [phi, psi], physical residual.
//   AD_PRECOND  psi only, preconditioning residual; also accumulates the adjoint of the
//               smeared sign (a.sb += R^ (1 - |q|)) and applies the sensor's VJP.
//   AD_SIGN     psi0 only: VJP of sgn = tanh(psi0 / max(|grad psi0|, delta_g)) for the
//               sign adjoint a.sb (no residual).
// Output: a.ub = own part of Y^; a.tb = trace adjoints pushed to the neighbours' - face
// slots; a.apart[block] += dL/dA contribution (physical mode).
// ------------------------------------------------------------------------------------
template <typename R, int D, int P, int MODE>
__global__ __launch_bounds__((AShape<D, P>::NT)) void k_adj_main(AJMain<R> a) {
    using S = AShape<D, P>;
    constexpr int N = S::N, NU = S::NU, NFA = S::NFA, EPB = S::EPB, NT = S::NT, G = S::GEO;
    constexpr int V = (MODE == AD_PHYS) ? 2 : 1;
    constexpr int NOPS = ops_size(N);
    constexpr bool RES = (MODE != AD_SIGN);          // a residual adjoint (not the sign VJP)
    constexpr bool SENS = (MODE == AD_PRECOND);
    constexpr int NPF = D * NFA;
    constexpr int NOW = 2 * NPF;                      // owned face items per element (+ then -)
    constexpr int XST = EPB * NU;
    constexpr int FI = (EPB * NOW + NT - 1) / NT;
    constexpr int I_OPS = (NOPS + NT - 1) / NT;
    constexpr int I_GEO = (EPB * G + NT - 1) / NT;
    constexpr int I_NBR = (EPB * 2 * D + NT - 1) / NT;
    constexpr int I_U = (EPB * NU + NT - 1) / NT;
    constexpr int I_NB = (EPB * NPF + NT - 1) / NT;
    using M = Math<R>;

    __shared__ R s_ops[NOPS];
    __shared__ R s_geo[EPB * G];
    __shared__ int s_nbr[EPB * 2 * D];
    __shared__ R s_u[V][EPB * NU];
    __shared__ R s_nb[V][EPB * NPF];
    __shared__ R s_q[V * D * XST];                    // forward q, then q~^
    __shared__ R s_d[RES ? V : 1][RES ? XST : 1];     // div^ = -R^/|J|
    __shared__ R s_fq[RES ? V * D : 1][RES ? EPB * NOW : 1];   // q_f^ at owned face points
    __shared__ R s_fu[RES ? V : 1][RES ? EPB * NOW : 1];       // u_L^ at owned face points
    __shared__ R s_fr[RES ? V : 1][RES ? EPB * NPF : 1];       // u_R^ at + face points
    __shared__ R s_x[SENS ? 3 : 1][SENS ? XST : 1];   // sensor: transform scratch and chi
    __shared__ R s_nu[EPB];
    __shared__ R s_nub[SENS ? XST + EPB * NOW : 1];   // sensor: nu^ contributions
    __shared__ R s_nue[EPB];                          // sensor: nu^ per element
    __shared__ double s_ab[NT];                       // dL/dA partial sums

    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    const int nel = (int)((a.E - e0) < EPB ? (a.E - e0) : EPB);
    const bool pt = tid < nel * NU;
    const int le = tid / NU;
    const int ip = tid - le * NU;
    const int64_t idx = (e0 + le) * NU + ip;
    int mi[D];
    {
        int r = ip;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            mi[k] = r % N;
            r /= N;
        }
    }
    double abar = 0.0;

    // ---- A: loads (all issued before the first wait) -----------------------------------
    R r_ops[I_OPS], r_geo[I_GEO], r_u[V][I_U], r_nb[I_NB][V];
    int32_t r_nbr[I_NBR];
#pragma unroll
    for (int j = 0; j < I_OPS; ++j) {
        const int i = tid + j * NT;
        r_ops[j] = (i < NOPS) ? a.ops[i] : R(0);
    }
#pragma unroll
    for (int j = 0; j < I_GEO; ++j) {
        const int i = tid + j * NT;
        r_geo[j] = (i < nel * G) ? a.geo[e0 * G + i] : R(0);
    }
#pragma unroll
    for (int j = 0; j < I_NBR; ++j) {
        const int i = tid + j * NT;
        r_nbr[j] = (i < nel * 2 * D) ? a.nbr[e0 * 2 * D + i] : -1;
    }
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
        for (int j = 0; j < I_U; ++j) {
            const int i = tid + j * NT;
            r_u[v][j] = (i < nel * NU) ? a.u[v][e0 * NU + i] : R(0);
        }
#pragma unroll
    for (int j = 0; j < I_NB; ++j) {
        const int it = tid + j * NT;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            // the forward traces are planar, [D][E][NFA]
            const int el = it / NPF, kf = (it - el * NPF) / NFA, tf = it - el * NPF - kf * NFA;
            r_nb[j][v] = (it < nel * NPF) ? a.Tp[v][((int64_t)kf * a.E + e0 + el) * NFA + tf] : R(0);
        }
    }
    R rb[V];
    R r_sg = R(0), r_sb = R(0);
    if (pt) {
        if constexpr (RES) {
#pragma unroll
            for (int v = 0; v < V; ++v) rb[v] = a.rbar[v][idx];
        }
        if constexpr (MODE != AD_PHYS) r_sg = a.sgn[idx];
        if constexpr (MODE == AD_SIGN) r_sb = a.sb[idx];
    }
    R r_gp[FI][V];
    if constexpr (RES) {
#pragma unroll
        for (int j = 0; j < FI; ++j) {
            const int it = tid + j * NT;
            const bool plus = it < nel * NPF;
#pragma unroll
            for (int v = 0; v < V; ++v) r_gp[j][v] = plus ? a.gp[v][e0 * NPF + it] : R(0);
        }
    }
#pragma unroll
    for (int j = 0; j < I_OPS; ++j)
        if (tid + j * NT < NOPS) s_ops[tid + j * NT] = r_ops[j];
#pragma unroll
    for (int j = 0; j < I_GEO; ++j)
        if (tid + j * NT < nel * G) s_geo[tid + j * NT] = r_geo[j];
#pragma unroll
    for (int j = 0; j < I_NBR; ++j)
        if (tid + j * NT < nel * 2 * D) s_nbr[tid + j * NT] = r_nbr[j];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
        for (int j = 0; j < I_U; ++j)
            if (tid + j * NT < nel * NU) s_u[v][tid + j * NT] = r_u[v][j];
#pragma unroll
    for (int j = 0; j < I_NB; ++j)
        if (tid + j * NT < nel * NPF)
#pragma unroll
            for (int v = 0; v < V; ++v) s_nb[v][tid + j * NT] = r_nb[j][v];
    __syncthreads();

    // ---- sensor forward: chi = V^-1 psi (kept for the VJP), energies, nu ----------------
    if constexpr (SENS) {
        const R* VI = &s_ops[op_vinv(N)];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const R* src = (k == 0) ? s_u[0] : s_x[(k - 1) & 1];
            R* dst = (k == D - 1) ? s_x[2] : s_x[k & 1];
            if (pt) {
                R acc = R(0);
                const int b0 = le * NU + ip - mi[k] * st<N>(k);
#pragma unroll
                for (int q = 0; q < N; ++q) acc += VI[mi[k] * N + q] * src[b0 + q * st<N>(k)];
                dst[tid] = acc;
            }
            __syncthreads();
        }
        if (tid < nel) {
            R ea = R(0), et = R(0);
            for (int i = 0; i < NU; ++i) {
                const R c = s_x[2][tid * NU + i];
                ea += c * c;
                int r = i, top = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    top |= ((r % N) == P);
                    r /= N;
                }
                if (top) et += c * c;
            }
            s_nu[tid] = visc_ramp(ea, et, a.ph.s0, a.ph.kappa, a.ph.nu_max);
        }
        __syncthreads();
    }

    // ---- B: forward corrected gradient q (Steps 1-3) and div^ --------------------------
    R q[V][D];
    if (pt) {
        const R* gg = &s_geo[le * G];
        const R* Ji = gg + D + D * D;
        const R* cp = &s_ops[op_cp(N)];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            R qt[D];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const bool hk = s_nbr[le * 2 * D + 2 * k + 1] >= 0;
                const R* Dk = &s_ops[hk ? op_dt(N) : OP_D1] + mi[k] * N;
                const int b0 = le * NU + ip - mi[k] * st<N>(k);
                R acc = R(0);
#pragma unroll
                for (int b = 0; b < N; ++b) acc += Dk[b] * s_u[v][b0 + b * st<N>(k)];
                acc += cp[mi[k]] * s_nb[v][le * NPF + k * NFA + tang_index<D, N>(k, mi)];
                qt[k] = acc;
            }
#pragma unroll
            for (int i = 0; i < D; ++i) {
                R acc = R(0);
#pragma unroll
                for (int k = 0; k < D; ++k) acc += Ji[k * D + i] * qt[k];
                q[v][i] = acc;
                s_q[(v * D + i) * XST + tid] = acc;
            }
            if constexpr (RES) s_d[v][tid] = -rb[v] / gg[D + 2 * D * D];
        }
    }
    __syncthreads();

    // ---- C: pointwise VJPs at solution points and face VJPs ----------------------------
    R ub[V], qb[V][D];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        ub[v] = R(0);
#pragma unroll
        for (int i = 0; i < D; ++i) qb[v][i] = R(0);
    }
    if (pt) {
        const R* gg = &s_geo[le * G];
        const R det = gg[D + 2 * D * D];
        const R* Ji = gg + D + D * D;
        if constexpr (RES) {
            // f~^_k = DH_k^T div^ along the line; f^ = |J| J^-T f~^
            const R* DH = &s_ops[op_dh(N)];
            R fb[V][D];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R ftb[D];
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const int b0 = le * NU + ip - mi[k] * st<N>(k);
                    R acc = R(0);
#pragma unroll
                    for (int b = 0; b < N; ++b) acc += DH[b * N + mi[k]] * s_d[v][b0 + b * st<N>(k)];
                    ftb[k] = acc;
                }
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    R acc = R(0);
#pragma unroll
                    for (int k = 0; k < D; ++k) acc += Ji[k * D + i] * ftb[k];
                    fb[v][i] = det * acc;
                }
            }
            if constexpr (MODE == AD_PHYS) {
                const R* xi = &s_ops[op_xi(N)];
                R x[D], vu[D];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    R acc = gg[i];
#pragma unroll
                    for (int j = 0; j < D; ++j) acc += gg[D + i * D + j] * (xi[mi[j]] + R(1));
                    x[i] = acc;
                }
                Phys<R> pu = a.ph;
                pu.ampg = a.gt;                        // unit-amplitude field g(t) v0(x)
                velocity<R, D>(pu, x, vu);
                const R A = a.amp;
                R vel[D], v2 = R(0), g2 = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    vel[i] = A * vu[i];
                    v2 += vel[i] * vel[i];
                    g2 += q[1][i] * q[1][i];
                }
                const R vm = M::sqrt_(v2);
                const bool act = vm > a.ph.gamma;
                const R mm = act ? vm : a.ph.gamma;
                const R rn = M::rsqrt_(g2 + a.ph.delta_n * a.ph.delta_n);
                const R phi = s_u[0][tid], psi = s_u[1][tid];
                const R pp = phi * (R(1) - phi);
                const R sharp = a.ph.gamma * pp * rn;
                R w = R(0), fdv = R(0), fdq0 = R(0), fdq1 = R(0), f1v = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    w += fb[0][i] * q[1][i];
                    fdv += fb[0][i] * vel[i];
                    fdq0 += fb[0][i] * q[0][i];
                    f1v += fb[1][i] * vel[i];
                }
                // f0 = phi v - mm (eps q0 - gamma phi (1-phi) rn q1);  f1 = psi v
                ub[0] = fdv + mm * a.ph.gamma * (R(1) - R(2) * phi) * rn * w;
                ub[1] = f1v;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    qb[0][i] = -mm * a.ph.eps * fb[0][i];
                    qb[1][i] = mm * sharp * fb[0][i] - mm * a.ph.gamma * pp * rn * rn * rn * q[1][i] * w;
                }
                // dL/dA: v = A g v0, mm = max(gamma, |v|)
                R fdu0 = R(0), fdu1 = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    fdu0 += fb[0][i] * vu[i];
                    fdu1 += fb[1][i] * vu[i];
                }
                R dmm = R(0);
                if (act) {
                    R vu2 = R(0);
#pragma unroll
                    for (int i = 0; i < D; ++i) vu2 += vu[i] * vu[i];
                    dmm = (A >= R(0) ? R(1) : R(-1)) * M::sqrt_(vu2);
                }
                abar += (double)(phi * fdu0 - dmm * (a.ph.eps * fdq0 - sharp * w) + psi * fdu1);
            }
            if constexpr (MODE == AD_PRECOND) {
                // g = -nu q;  S = sgn (1 - |q|)
                const R nu = s_nu[le];
                R g2 = R(0), qdg = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    g2 += q[0][i] * q[0][i];
                    qdg += q[0][i] * fb[0][i];
                }
                const R qm = M::sqrt_(g2);
                a.sb[idx] += rb[0] * (R(1) - qm);
                const R sq = (qm > R(0)) ? -r_sg * rb[0] / qm : R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) qb[0][i] = -nu * fb[0][i] + sq * q[0][i];
                s_nub[tid] = -qdg;                          // nu^ contribution of this point
            }
        }
        if constexpr (MODE == AD_SIGN) {
            // sgn = tanh(psi0 / gm), gm = max(|q|, delta_g)
            R g2 = R(0);
#pragma unroll
            for (int i = 0; i < D; ++i) g2 += q[0][i] * q[0][i];
            const R qm = M::sqrt_(g2);
            const bool act = qm > a.ph.delta_g;
            const R gm = act ? qm : a.ph.delta_g;
            const R psi0 = s_u[0][tid];
            const R sg = M::tanh_(psi0 / gm);
            const R dz = r_sb * (R(1) - sg * sg);          // d/d(psi0/gm)
            ub[0] = dz / gm;
            if (act) {
                const R c = -dz * psi0 / (gm * gm * qm);
#pragma unroll
                for (int i = 0; i < D; ++i) qb[0][i] = c * q[0][i];
            }
        }
    } else if constexpr (SENS) {
        if (tid < XST) s_nub[tid] = R(0);
    }

    if constexpr (RES) {
        // owned face points: + faces [0, nel*NPF) and boundary - faces [nel*NPF, 2 nel NPF)
#pragma unroll
        for (int j = 0; j < FI; ++j) {
            const int it = tid + j * NT;
            if (it >= EPB * NOW) continue;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                s_fu[v][it] = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) s_fq[v * D + i][it] = R(0);
            }
            if constexpr (SENS) s_nub[XST + it] = R(0);
            if (it >= 2 * nel * NPF) continue;
            const bool plus = it < nel * NPF;
            const int itf = plus ? it : it - nel * NPF;
            const int el = itf / NPF, r = itf - el * NPF, k = r / NFA, t = r - k * NFA;
            const int s = plus ? 1 : 0;
            const int32_t en = s_nbr[el * 2 * D + 2 * k + s];
            if (plus) {
#pragma unroll
                for (int v = 0; v < V; ++v) s_fr[v][itf] = R(0);
            }
            if (!plus && en >= 0) continue;
            const int base = el * NU + face_base<D, N>(k, t);
            const R* l = &s_ops[s ? op_lp(N) : op_lm(N)];
            const R* lc = &s_ops[s ? op_cp(N) : op_cm(N)];
            const R* gg = &s_geo[el * G];
            const R* Ji = gg + D + D * D;
            const R det_e = gg[D + 2 * D * D];
            R mag2 = R(0);
#pragma unroll
            for (int i = 0; i < D; ++i) mag2 += Ji[k * D + i] * Ji[k * D + i];
            const R mag = M::sqrt_(mag2);
            R nrm[D];
#pragma unroll
            for (int i = 0; i < D; ++i) nrm[i] = (s ? R(1) : R(-1)) * Ji[k * D + i] / mag;
            const R sc = det_e * mag;
            // forward face quantities
            R uL[V], uR[V], qf[V][D], Fb[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R acc = R(0), db = R(0);
#pragma unroll
                for (int qq = 0; qq < N; ++qq) {
                    acc += l[qq] * s_u[v][base + qq * st<N>(k)];
                    db += lc[qq] * s_d[v][base + qq * st<N>(k)];
                }
                uL[v] = acc;
                uR[v] = (en >= 0) ? s_nb[v][el * NPF + k * NFA + t] : acc;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    R qa = R(0);
#pragma unroll
                    for (int qq = 0; qq < N; ++qq) qa += l[qq] * s_q[(v * D + i) * XST + base + qq * st<N>(k)];
                    qf[v][i] = qa;
                }
                // adjoint of the stored (scaled) flux: own lifting + the neighbour's push
                Fb[v] = sc * (db + (plus ? r_gp[j][v] : R(0)));
            }
            R uLb[V], uRb[V], qfb[V][D];
            if constexpr (MODE == AD_PHYS) {
                const R* xi = &s_ops[op_xi(N)];
                R x[D];
                {
                    int tt = t;
                    R xr[D];
#pragma unroll
                    for (int m = 0; m < D; ++m) {
                        if (m == k) {
                            xr[m] = s ? R(2) : R(0);
                        } else {
                            xr[m] = xi[tt % N] + R(1);
                            tt /= N;
                        }
                    }
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        R acc = gg[i];
#pragma unroll
                        for (int m = 0; m < D; ++m) acc += gg[D + i * D + m] * xr[m];
                        x[i] = acc;
                    }
                }
                Phys<R> pu = a.ph;
                pu.ampg = a.gt;
                R vu[D];
                velocity<R, D>(pu, x, vu);
                const R A = a.amp;
                R v2 = R(0), vn = R(0), vun = R(0), g2 = R(0), qn0 = R(0), qn1 = R(0), vu2 = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const R vi = A * vu[i];
                    v2 += vi * vi;
                    vu2 += vu[i] * vu[i];
                    vn += vi * nrm[i];
                    vun += vu[i] * nrm[i];
                    g2 += qf[1][i] * qf[1][i];
                    qn0 += qf[0][i] * nrm[i];
                    qn1 += qf[1][i] * nrm[i];
                }
                const R vm = M::sqrt_(v2);
                const bool act = vm > a.ph.gamma;
                const R mm = act ? vm : a.ph.gamma;
                const R rn = M::rsqrt_(g2 + a.ph.delta_n * a.ph.delta_n);
                const R pL = uL[0], pR = uR[0], sL = uL[1], sR = uR[1];
                const R pp = pL * (R(1) - pL);
                const R F0b = Fb[0], F1b = Fb[1];
                const R tau = a.ph.tau;
                uLb[0] = F0b * (R(0.5) * vn + tau + mm * a.ph.gamma * (R(1) - R(2) * pL) * qn1 * rn);
                uRb[0] = F0b * (R(0.5) * vn - tau);
                uLb[1] = F1b * (R(0.5) * vn + tau);
                uRb[1] = F1b * (R(0.5) * vn - tau);
                const R cq = F0b * mm * a.ph.gamma * pp;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    qfb[0][i] = -F0b * mm * a.ph.eps * nrm[i];
                    qfb[1][i] = cq * (nrm[i] * rn - qn1 * rn * rn * rn * qf[1][i]);
                }
                const R dmm = act ? (A >= R(0) ? R(1) : R(-1)) * M::sqrt_(vu2) : R(0);
                abar += (double)(F0b * (R(0.5) * (pL + pR) * vun
                                        - dmm * (a.ph.eps * qn0 - a.ph.gamma * pp * qn1 * rn))
                                 + F1b * R(0.5) * (sL + sR) * vun);
            } else {
                // G = -nu q.n + tau (psi_L - psi_R)
                const R nu = s_nu[el];
                R qn = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) qn += qf[0][i] * nrm[i];
                uLb[0] = a.ph.tau * Fb[0];
                uRb[0] = -a.ph.tau * Fb[0];
#pragma unroll
                for (int i = 0; i < D; ++i) qfb[0][i] = -nu * Fb[0] * nrm[i];
                s_nub[XST + it] = -qn * Fb[0];
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const R ghost = (en >= 0) ? R(0) : uRb[v];   // ghost state = interior state
                s_fu[v][it] = uLb[v] + ghost;
#pragma unroll
                for (int i = 0; i < D; ++i) s_fq[v * D + i][it] = qfb[v][i];
                if (plus && en >= 0) s_fr[v][itf] = uRb[v];
            }
        }
    }
    s_ab[tid] = abar;
    __syncthreads();

    // ---- D: gather face adjoints to the solution points; q~^ = J^-1 q^ -> LDS ---------
    if (pt) {
        const R* gg = &s_geo[le * G];
        const R* Ji = gg + D + D * D;
        if constexpr (RES) {
            const R* lp = &s_ops[op_lp(N)];
            const R* lm = &s_ops[op_lm(N)];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int tk = tang_index<D, N>(k, mi);
                // + face of this line (always owned)
                const int ip_ = le * NPF + k * NFA + tk;
                // - face of this line (owned only on a boundary)
                const int im_ = nel * NPF + le * NPF + k * NFA + tk;
                const bool bm = s_nbr[le * 2 * D + 2 * k] < 0;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    ub[v] += lp[mi[k]] * s_fu[v][ip_];
                    if (bm) ub[v] += lm[mi[k]] * s_fu[v][im_];
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        qb[v][i] += lp[mi[k]] * s_fq[v * D + i][ip_];
                        if (bm) qb[v][i] += lm[mi[k]] * s_fq[v * D + i][im_];
                    }
                }
            }
        }
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int k = 0; k < D; ++k) {
                R acc = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) acc += Ji[k * D + i] * qb[v][i];
                s_q[(v * D + k) * XST + tid] = acc;           // q~^ (forward q no longer used)
            }
    }
    if constexpr (SENS) {
        // nu^ of each element: its points and its owned face points, in a fixed order
        if (tid < nel) {
            R acc = R(0);
            for (int i = 0; i < NU; ++i) acc += s_nub[tid * NU + i];
            for (int i = 0; i < NPF; ++i) acc += s_nub[XST + tid * NPF + i];
            for (int i = 0; i < NPF; ++i) acc += s_nub[XST + nel * NPF + tid * NPF + i];
            s_nue[tid] = acc;
        }
    }
    if (tid == 0) {
        double acc = 0.0;
        for (int i = 0; i < NT; ++i) acc += s_ab[i];
        if (MODE == AD_PHYS) a.apart[blockIdx.x] += acc;
    }
    __syncthreads();

    // ---- E: transposed gradient; trace adjoints pushed to the neighbours --------------
    if (pt) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const bool hk = s_nbr[le * 2 * D + 2 * k + 1] >= 0;
            const R* Dk = &s_ops[hk ? op_dt(N) : OP_D1];
            const int b0 = le * NU + ip - mi[k] * st<N>(k);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R acc = R(0);
#pragma unroll
                for (int b = 0; b < N; ++b) acc += Dk[b * N + mi[k]] * s_q[(v * D + k) * XST + b0 + b * st<N>(k)];
                ub[v] += acc;
            }
        }
    }
    // + faces with a neighbour: nb^ = sum_a cp[a] q~^_k(line a), plus the flux's u_R^
#pragma unroll
    for (int j = 0; j < I_NB; ++j) {
        const int it = tid + j * NT;
        if (it >= nel * NPF) continue;
        const int el = it / NPF, r = it - el * NPF, k = r / NFA, t = r - k * NFA;
        const int32_t en = s_nbr[el * 2 * D + 2 * k + 1];
        if (en < 0) continue;
        const int base = el * NU + face_base<D, N>(k, t);
        const R* cp = &s_ops[op_cp(N)];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            R acc = R(0);
#pragma unroll
            for (int qq = 0; qq < N; ++qq) acc += cp[qq] * s_q[(v * D + k) * XST + base + qq * st<N>(k)];
            if constexpr (RES) acc += s_fr[v][it];
            a.tb[v][((int64_t)en * D + k) * NFA + t] = acc;
        }
    }

    // ---- sensor VJP: nu^ -> s^ -> chi^ -> psi^ += V^-T chi^ -----------------------------
    if constexpr (SENS) {
        // s_x[2] holds chi; s_x[0], s_x[1] are scratch
        __syncthreads();
        // per-element derivative factors, one thread per element
        if (tid < nel) {
            R ea = R(0), et = R(0);
            for (int i = 0; i < NU; ++i) {
                const R c = s_x[2][tid * NU + i];
                ea += c * c;
                int r = i, top = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    top |= ((r % N) == P);
                    r /= N;
                }
                if (top) et += c * c;
            }
            R fa = R(0), ft = R(0);
            if (ea > R(0) && et > R(0)) {
                const R sv = M::log10_(et / ea);
                const R s0 = a.ph.s0, kap = a.ph.kappa;
                if (sv >= s0 - kap && sv <= s0 + kap) {
                    // nu = nu_max/2 (1 + sin(pi (s - s0) / (2 kappa)))
                    const R arg = (sv - s0) / (R(2) * kap);
                    R sn, cs;
                    M::sincospi_(arg, &sn, &cs);
                    const R dnu = R(0.5) * a.ph.nu_max * cs * R(M_PI) / (R(2) * kap);
                    const R sbar = s_nue[tid] * dnu / R(M_LN10);
                    ft = sbar / et;
                    fa = -sbar / ea;
                }
            }
            s_x[0][tid * NU] = fa;       // element factors (slot 0 of the element's range)
            s_x[1][tid * NU] = ft;
        }
        __syncthreads();
        R chib = R(0);
        if (pt) {
            const R fa = s_x[0][le * NU], ft = s_x[1][le * NU];
            int top = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) top |= (mi[k] == P);
            chib = R(2) * s_x[2][tid] * (fa + (top ? ft : R(0)));
        }
        __syncthreads();
        if (pt) s_x[0][tid] = chib;
        __syncthreads();
        // psi^ += (V^-1 (x) ... )^T chi^: one transposed 1D transform per direction
        const R* VI = &s_ops[op_vinv(N)];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const R* src = s_x[k & 1];
            R* dst = s_x[(k + 1) & 1];
            R acc = R(0);
            if (pt) {
                const int b0 = le * NU + ip - mi[k] * st<N>(k);
#pragma unroll
                for (int q2 = 0; q2 < N; ++q2) acc += VI[q2 * N + mi[k]] * src[b0 + q2 * st<N>(k)];
            }
            __syncthreads();
            if (pt) dst[tid] = acc;
            __syncthreads();
        }
        if (pt) ub[0] += s_x[D & 1][tid];
    }

    if (pt) {
#pragma unroll
        for (int v = 0; v < V; ++v) a.ub[v][idx] = ub[v];
    }
}

// ------------------------------------------------------------------------------------
// k_adj_finish: Y^ = ub + sum over - faces with an owner of lm (x) tb; then the reverse
// RK4 combine:  ya += Y^;  next R^ = c_prev * yb + c_cur * Y^  (when c_prev or c_cur set)
// ------------------------------------------------------------------------------------
template <typename R, int D, int P, int V>
__global__ __launch_bounds__((AShape<D, P>::NT)) void k_adj_finish(AJFinish<R> a) {
    using S = AShape<D, P>;
    constexpr int N = S::N, NU = S::NU, NFA = S::NFA, EPB = S::EPB, NT = S::NT, G = S::GEO;
    constexpr int I_T = (EPB * D * NFA + NT - 1) / NT;
    __shared__ R s_lm[N];
    __shared__ R s_cm[N];
    __shared__ int s_nbr[EPB * 2 * D];
    __shared__ R s_r[V][EPB * NU];
    __shared__ R s_y[V][EPB * NU];
    __shared__ R s_det[EPB];
    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    const int nel = (int)((a.E - e0) < EPB ? (a.E - e0) : EPB);
    const bool pt = tid < nel * NU;
    const bool push = a.ynext[0] != nullptr;
    const int le = tid / NU;
    const int ip = tid - le * NU;
    const int64_t idx = (e0 + le) * NU + ip;
    const R r_l = (tid < N) ? a.ops[op_lm(N) + tid] : R(0);
    int32_t r_n[(EPB * 2 * D + NT - 1) / NT];
#pragma unroll
    for (int j = 0; j < (EPB * 2 * D + NT - 1) / NT; ++j) {
        const int i = tid + j * NT;
        r_n[j] = (i < nel * 2 * D) ? a.nbr[e0 * 2 * D + i] : -1;
    }
    // inputs of the next stage's push
    int32_t r_own[I_T];
    R r_y[V];
    if (push) {
        owners_of_minus_faces<R, D, P, V>(r_own, a.nbr, e0, nel, tid);
#pragma unroll
        for (int v = 0; v < V; ++v) r_y[v] = pt ? a.ynext[v][idx] : R(0);
        const R r_c = (tid < N) ? a.ops[op_cm(N) + tid] : R(0);
        const R r_d = (tid < nel) ? a.geo[(e0 + tid) * G + D + 2 * D * D] : R(1);
        if (tid < N) s_cm[tid] = r_c;
        if (tid < nel) s_det[tid] = r_d;
    }
    if (tid < N) s_lm[tid] = r_l;
#pragma unroll
    for (int j = 0; j < (EPB * 2 * D + NT - 1) / NT; ++j)
        if (tid + j * NT < nel * 2 * D) s_nbr[tid + j * NT] = r_n[j];
    __syncthreads();
    if (pt) {
        int mi[D];
        {
            int r = ip;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                mi[k] = r % N;
                r /= N;
            }
        }
        // explicit fused multiply-adds: the rounding does not depend on what the surrounding
        // code lets the compiler contract
        using M = Math<R>;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            R y = a.ub[v][idx];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                if (s_nbr[le * 2 * D + 2 * k] < 0) continue;
                const int tk = tang_index<D, N>(k, mi);
                y = M::fma_(s_lm[mi[k]], a.tb[v][((e0 + le) * D + k) * NFA + tk], y);
            }
            if (a.ya[v]) a.ya[v][idx] += y;
            if (a.rnext[v]) {
                const R rn = M::fma_(a.c_cur, y, a.c_prev * a.yb[v][idx]);
                a.rnext[v][idx] = rn;
                if (push) {
                    s_r[v][tid] = rn;
                    s_y[v][tid] = r_y[v];
                }
            }
        }
    }
    if (!push) return;
    // the push of the next stage: its R^ is rnext of this block's own points
    __syncthreads();
    const R* sr[V];
    const R* sy[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        sr[v] = s_r[v];
        sy[v] = s_y[v];
    }
    push_minus_faces<R, D, P, V>(s_cm, s_lm, sr, sy, s_det, r_own, a.gp, a.Tp, nel, tid, a.E);
}

// elementwise helpers of the reverse sweep

// adjoint of the reset psi0 = phi - 1/2 (LINEAR) or eps_w ln(c / (1 - c)) (LOGIT):
// phi^ += psi0^ dpsi0/dphi
template <typename R>
__global__ void k_reset_adj(R* phib, const R* psi0b, const R* phi, int64_t n, int mode,
                            double eps_w, double dphi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (mode == PCPF_RESET_LOGIT) {
        const double c = (double)phi[i];
        if (c > dphi && c < 1.0 - dphi) phib[i] += (R)((double)psi0b[i] * eps_w / (c * (1.0 - c)));
    } else {
        phib[i] += psi0b[i];
    }
}

template <typename R>
__global__ void k_loss_seed(R* out, const R* phi, const R* target, const R* geo, const R* w,
                            int64_t E, int nu, int n, int d, int geo_stride) {
    // dL/dphi for L = 1/2 sum |J| W (phi - target)^2 (helper for tests and examples)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E * nu) return;
    const int64_t e = i / nu;
    int r = (int)(i - e * nu);
    R W = R(1);
    for (int k = 0; k < d; ++k) {
        W *= w[r % n];
        r /= n;
    }
    out[i] = geo[e * geo_stride + d + 2 * d * d] * W * (phi[i] - target[i]);
}

template <typename R, int D, int P>
struct AImpl {
    using S = AShape<D, P>;
    static unsigned grid(int64_t E) { return (unsigned)((E + S::EPB - 1) / S::EPB); }
    static void push(int nvar, const AJPush<R>& a, hipStream_t st) {
        const dim3 g(grid(a.E)), b(S::NT);
        if (nvar == 2) hipLaunchKernelGGL((k_adj_push<R, D, P, 2>), g, b, 0, st, a);
        else hipLaunchKernelGGL((k_adj_push<R, D, P, 1>), g, b, 0, st, a);
    }
    static void main(int mode, const AJMain<R>& a, hipStream_t st) {
        const dim3 g(grid(a.E)), b(S::NT);
        if (mode == AD_PHYS) hipLaunchKernelGGL((k_adj_main<R, D, P, AD_PHYS>), g, b, 0, st, a);
        else if (mode == AD_PRECOND) hipLaunchKernelGGL((k_adj_main<R, D, P, AD_PRECOND>), g, b, 0, st, a);
        else hipLaunchKernelGGL((k_adj_main<R, D, P, AD_SIGN>), g, b, 0, st, a);
    }
    static void finish(int nvar, const AJFinish<R>& a, hipStream_t st) {
        const dim3 g(grid(a.E)), b(S::NT);
        if (nvar == 2) hipLaunchKernelGGL((k_adj_finish<R, D, P, 2>), g, b, 0, st, a);
        else hipLaunchKernelGGL((k_adj_finish<R, D, P, 1>), g, b, 0, st, a);
    }
};

template <typename R, int D, int P>
bool afill(AdjLaunchers<R>* L) {
    L->epb = AShape<D, P>::EPB;
    L->push = &AImpl<R, D, P>::push;
    L->main = &AImpl<R, D, P>::main;
    L->finish = &AImpl<R, D, P>::finish;
    return true;
}

}  // namespace

template <typename R>
bool get_adj_launchers(int d, int p, AdjLaunchers<R>* L) {
    if (d == 2) {
        switch (p) {
            case 1: return afill<R, 2, 1>(L);
            case 2: return afill<R, 2, 2>(L);
            case 3: return afill<R, 2, 3>(L);
            case 4: return afill<R, 2, 4>(L);
            case 5: return afill<R, 2, 5>(L);
            case 6: return afill<R, 2, 6>(L);
            default: return false;
        }
    }
    if (d == 3) {
        switch (p) {
            case 1: return afill<R, 3, 1>(L);
            case 2: return afill<R, 3, 2>(L);
            case 3: return afill<R, 3, 3>(L);
            case 4: return afill<R, 3, 4>(L);
            case 5: return afill<R, 3, 5>(L);
            default: return false;
        }
    }
    return false;
}
template bool get_adj_launchers<double>(int, int, AdjLaunchers<double>*);
template bool get_adj_launchers<float>(int, int, AdjLaunchers<float>*);


template <typename R>
void launch_reset_adj(R* phib, const R* psi0b, const R* phi, int64_t n, int mode, double eps_w,
                      double dphi, hipStream_t s) {
    hipLaunchKernelGGL((k_reset_adj<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, phib,
                       psi0b, phi, n, mode, eps_w, dphi);
}
template void launch_reset_adj<double>(double*, const double*, const double*, int64_t, int, double, double, hipStream_t);
template void launch_reset_adj<float>(float*, const float*, const float*, int64_t, int, double, double, hipStream_t);

template <typename R>
void launch_loss_seed(R* out, const R* phi, const R* target, const R* geo, const R* w, int64_t E,
                      int nu, int n, int d, hipStream_t s) {
    const int64_t tot = E * nu;
    hipLaunchKernelGGL((k_loss_seed<R>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, out,
                       phi, target, geo, w, E, nu, n, d, d + 2 * d * d + 1);
}
template void launch_loss_seed<double>(double*, const double*, const double*, const double*, const double*, int64_t, int, int, int, hipStream_t);
template void launch_loss_seed<float>(float*, const float*, const float*, const float*, const float*, int64_t, int, int, int, hipStream_t);

}  // namespace pcpf
