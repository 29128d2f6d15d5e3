// HIP kernels of the FR-PCPF residual on triangles (gfx950): dense per-element operators.
//
// The triangle element of order p has N_u = (p+1)(p+2)/2 solution points and N_f = 3(p+1)
// flux points (p+1 on each edge); its operators (§3.1: interpolation M0, derivatives D_k,
// the correction-function lifting Lift, the modal transform of the sensor) are dense
// N_f x N_u / N_u x N_u / N_u x N_f matrices applied per element. A block holds
// EPB = floor(256 / max(N_u, N_f)) elements, one thread per solution point for the point
// work and one thread per flux point for the face work, with the element data and the
// operator block in LDS.
//
// Face coupling goes through a per-flux-point table: slot[e N_f + f] = 2 s' + o, where s'
// is the coincident flux point of the neighbouring element and o = 1 when this element
// owns the face (computes its common flux, LDG beta = +1/2); -1 on a boundary (ghost state
// B(u) = u, B(q) = q of §3.3, the element's own flux). Every element writes the traces of
// its own flux points (Tf) and reads its partner's through the table; the owner writes the
// physical common normal flux F . n into its own slot (Fs) and the other element reads it,
// negated (its outward normal is opposite). Each side scales it by its own |J| |J^-T nhat|:
// the two sides of an edge generally map onto reference edges of different lengths (a leg
// on one side, the hypotenuse on the other), so their transformed fluxes are not opposite.
#include <hip/hip_ext.h>

#include <type_traits>

#include "pcpf_device.h"
#include "pcpf_internal.h"
#include "pcpf_tri.h"

namespace pcpf {
namespace {

using namespace dev;

// grad_flux on triangles, all four modes of k_grad_flux (physical, preconditioning, sign,
// sensor).
template <typename R, int P, int MODE, bool NPHI>
__global__ __launch_bounds__(256) void k_tri_grad_flux(GFArgs<R> a) {
    using S = TriShape<P>;
    constexpr int NU = S::NU, NF = S::NF, EPB = S::EPB, G = S::G;
    constexpr int V = (MODE == GF_PHYS) ? 2 : 1;
    constexpr int NV = NPHI ? 0 : V - 1;
    constexpr int NOPS = S::ODH0;             // the operators up to the normals (no DH_k)
    constexpr bool FLUX = (MODE == GF_PHYS || MODE == GF_PRECOND);
    constexpr bool SENS = (MODE == GF_PRECOND || MODE == GF_SENSOR);
    constexpr bool GRAD = (MODE != GF_SENSOR);
    constexpr int XU = EPB * NU, XF = EPB * NF;
    using M = Math<R>;

    __shared__ R s_ops[NOPS];
    __shared__ R s_geo[EPB * G];
    __shared__ R s_u[V][XU];
    __shared__ R s_tr[V][XF];                 // own traces
    __shared__ R s_jn[GRAD ? V * 2 : 1][XF];  // nhat_k (common - own) at the flux points
    __shared__ R s_q[GRAD ? V * 2 : 1][XU];   // physical gradient
    __shared__ R s_f[FLUX ? V * 2 : 1][XU];   // transformed flux at the solution points
    __shared__ R s_fp[FLUX ? V : 1][XF];      // its discontinuous normal component
    __shared__ R s_chi[SENS ? XU : 1];
    __shared__ R s_nu[EPB];
    __shared__ int s_slot[XF];

    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    const int nel = (int)((a.E - e0) < EPB ? (a.E - e0) : EPB);
    const bool pt = tid < nel * NU;
    const bool fp = tid < nel * NF;
    const int pe = tid / NU, pi = tid - pe * NU;          // point thread: element, point
    const int fe = tid / NF, fi = tid - fe * NF;          // flux-point thread: element, point
    const R* M0 = &s_ops[S::OM0];
    const R* Dm[2] = {&s_ops[S::OD0], &s_ops[S::OD1]};
    const R* LF = &s_ops[S::OL];
    const R* UR = &s_ops[S::OUR];
    const R* FR = &s_ops[S::OFR];
    const R* NH = &s_ops[S::ONH];

    // ---- A: loads -------------------------------------------------------------------
    for (int i = tid; i < NOPS; i += 256) s_ops[i] = a.ops[i];
    for (int i = tid; i < nel * G; i += 256) s_geo[i] = a.geo[e0 * G + i];
    for (int v = 0; v < V; ++v) {
        if (pt) s_u[v][tid] = a.u[v][e0 * NU + tid];
    }
    int code = -1;
    R ptr[V];
    if (fp) {
        code = a.nbr[e0 * NF + tid];
        s_slot[tid] = code;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            s_tr[v][tid] = a.Tp[v][e0 * NF + tid];
            ptr[v] = code >= 0 ? a.Tp[v][code >> 1] : R(0);
        }
    }
    __syncthreads();

    // ---- sensor (§3.2): modal coefficients, energies per element --------------------------
    if constexpr (SENS) {
        const R* VI = &s_ops[S::OVI];
        const R* TOP = &s_ops[S::OTOP];
        if (pt) {
            R c = R(0);
            for (int j = 0; j < NU; ++j) c += VI[pi * NU + j] * s_u[0][pe * NU + j];
            s_chi[tid] = c;
        }
        __syncthreads();
        if (tid < nel) {
            R ea = R(0), et = R(0);
            for (int j = 0; j < NU; ++j) {
                const R c = s_chi[tid * NU + j];
                ea += c * c;
                if (TOP[j] != R(0)) et += c * c;
            }
            const R nu = visc_ramp(ea, et, a.ph.s0, a.ph.kappa, a.ph.nu_max);
            s_nu[tid] = nu;
            if constexpr (MODE == GF_SENSOR) a.out[e0 + tid] = nu;
        }
        __syncthreads();
        if constexpr (MODE == GF_SENSOR) return;
    }

    if constexpr (GRAD) {
        // ---- B1: LDG jumps (Step 2): the owner takes the neighbour's trace --------------
        if (fp) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const R jump = (code >= 0 && (code & 1)) ? ptr[v] - s_tr[v][tid] : R(0);
                s_jn[v * 2 + 0][tid] = NH[fi * 2 + 0] * jump;
                s_jn[v * 2 + 1][tid] = NH[fi * 2 + 1] * jump;
            }
        }
        __syncthreads();

        // ---- B2: corrected gradient (Step 3) and fluxes at the solution points (Step 4) --
        R Sdet = R(0);
        if (pt) {
            const R* gg = &s_geo[pe * G];
            const R det = gg[2 + 8];
            const R* Ji = gg + 2 + 4;              // Jinv[k][i] = Ji[k*2 + i]
            R q[V][2];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R qt[2];
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    R acc = R(0);
                    for (int j = 0; j < NU; ++j) acc += Dm[k][pi * NU + j] * s_u[v][pe * NU + j];
                    for (int f = 0; f < NF; ++f) acc += LF[pi * NF + f] * s_jn[v * 2 + k][pe * NF + f];
                    qt[k] = acc;
                }
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    q[v][i] = Ji[0 * 2 + i] * qt[0] + Ji[1 * 2 + i] * qt[1];
                    s_q[v * 2 + i][tid] = q[v][i];
                }
            }
            if constexpr (MODE == GF_SIGN) {
                R g = M::sqrt_(q[0][0] * q[0][0] + q[0][1] * q[0][1]);
                if (!(g > a.ph.delta_g)) g = a.ph.delta_g;
                a.out[e0 * NU + tid] = M::tanh_(s_u[0][tid] / g);
            }
            if constexpr (MODE == GF_PHYS) {
                R x[2], vel[2];
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    x[i] = gg[i] + gg[2 + i * 2 + 0] * UR[pi * 2 + 0] + gg[2 + i * 2 + 1] * UR[pi * 2 + 1];
                velocity<R, 2>(a.ph, x, vel);
                const R v2 = vel[0] * vel[0] + vel[1] * vel[1];
                const R g2 = q[NV][0] * q[NV][0] + q[NV][1] * q[NV][1];
                const R mm = max_sqrt(v2, a.ph.gamma);
                const R rn = M::rsqrt_(g2 + a.ph.delta_n * a.ph.delta_n);
                const R phi = s_u[0][tid], psi = s_u[1][tid];
                const R sharp = a.ph.gamma * phi * (R(1) - phi) * rn;
                R f0[2], f1[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const R fvis = mm * (a.ph.eps * q[0][i] - sharp * q[NV][i]);
                    f0[i] = phi * vel[i] - fvis;
                    f1[i] = psi * vel[i];
                }
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    s_f[0 * 2 + k][tid] = det * (Ji[k * 2 + 0] * f0[0] + Ji[k * 2 + 1] * f0[1]);
                    s_f[1 * 2 + k][tid] = det * (Ji[k * 2 + 0] * f1[0] + Ji[k * 2 + 1] * f1[1]);
                }
            }
            if constexpr (MODE == GF_PRECOND) {
                const R nu = s_nu[pe];
                const R g = M::sqrt_(q[0][0] * q[0][0] + q[0][1] * q[0][1]);
                R sg = a.sgn[e0 * NU + tid];
                if (a.sgn_current) {
                    R gd = g;
                    if (!(gd > a.ph.delta_g)) gd = a.ph.delta_g;
                    sg = M::tanh_(sg / gd);
                }
                Sdet = det * sg * (R(1) - g);
#pragma unroll
                for (int k = 0; k < 2; ++k)
                    s_f[k][tid] = -det * nu * (Ji[k * 2 + 0] * q[0][0] + Ji[k * 2 + 1] * q[0][1]);
            }
        }
        if constexpr (MODE == GF_SIGN) return;
        __syncthreads();

        // ---- C: discontinuous normal flux at every flux point; common normal flux at the
        // owned and boundary flux points (Step 5) -----------------------------------------
        if (fp) {
            const R* gg = &s_geo[fe * G];
            const R det = gg[2 + 8];
            const R* Ji = gg + 2 + 4;
            const R n0 = NH[fi * 2 + 0], n1 = NH[fi * 2 + 1];
            // f~perp = nhat . (M0 f~)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R a0 = R(0), a1 = R(0);
                for (int i = 0; i < NU; ++i) {
                    a0 += M0[fi * NU + i] * s_f[v * 2 + 0][fe * NU + i];
                    a1 += M0[fi * NU + i] * s_f[v * 2 + 1][fe * NU + i];
                }
                s_fp[v][tid] = n0 * a0 + n1 * a1;
            }
            if (code < 0 || (code & 1)) {
                // unit physical normal J^-T nhat / |J^-T nhat|
                R nr[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) nr[i] = Ji[0 * 2 + i] * n0 + Ji[1 * 2 + i] * n1;
                const R mag = M::sqrt_(nr[0] * nr[0] + nr[1] * nr[1]);
                nr[0] /= mag;
                nr[1] /= mag;
                R uL[V], uR[V], qn[V], g2 = R(0);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    uL[v] = s_tr[v][tid];
                    uR[v] = code >= 0 ? ptr[v] : uL[v];
                    R qa[2] = {R(0), R(0)};
                    for (int i = 0; i < NU; ++i) {
                        qa[0] += M0[fi * NU + i] * s_q[v * 2 + 0][fe * NU + i];
                        qa[1] += M0[fi * NU + i] * s_q[v * 2 + 1][fe * NU + i];
                    }
                    qn[v] = qa[0] * nr[0] + qa[1] * nr[1];
                    if (MODE == GF_PHYS && v == NV) g2 = qa[0] * qa[0] + qa[1] * qa[1];
                }
                const uint32_t slot = (uint32_t)(e0 * NF + tid);
                if constexpr (MODE == GF_PHYS) {
                    R x[2], vel[2];
#pragma unroll
                    for (int i = 0; i < 2; ++i)
                        x[i] = gg[i] + gg[2 + i * 2 + 0] * FR[fi * 2 + 0] + gg[2 + i * 2 + 1] * FR[fi * 2 + 1];
                    velocity<R, 2>(a.ph, x, vel);
                    const R v2 = vel[0] * vel[0] + vel[1] * vel[1];
                    const R vn = vel[0] * nr[0] + vel[1] * nr[1];
                    const R mm = max_sqrt(v2, a.ph.gamma);
                    const R rn = M::rsqrt_(g2 + a.ph.delta_n * a.ph.delta_n);
                    const R pL = uL[0], pR = uR[0], sL = uL[1], sR = uR[1];
                    const R fvn = mm * (a.ph.eps * qn[0] - a.ph.gamma * pL * (R(1) - pL) * qn[NV] * rn);
                    const R F0 = R(0.5) * (pL + pR) * vn - fvn + a.ph.tau * (pL - pR);
                    const R F1 = R(0.5) * (sL + sR) * vn + a.ph.tau * (sL - sR);
                    gst(a.Fp[0], slot, F0);
                    gst(a.Fp[1], slot, F1);
                } else {
                    const R F = -s_nu[fe] * qn[0] + a.ph.tau * (uL[0] - uR[0]);
                    gst(a.Fp[0], slot, F);
                }
            }
        }
        __syncthreads();

        // ---- E: volume part of Step 6: P = sum_k D_k f~_k - Lift f~perp (- |J| S) -----------
        if (pt) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R acc = R(0);
#pragma unroll
                for (int k = 0; k < 2; ++k)
                    for (int j = 0; j < NU; ++j) acc += Dm[k][pi * NU + j] * s_f[v * 2 + k][pe * NU + j];
                for (int f = 0; f < NF; ++f) acc -= LF[pi * NF + f] * s_fp[v][pe * NF + f];
                if constexpr (MODE == GF_PRECOND) acc -= Sdet;
                a.P[v][e0 * NU + tid] = acc;
            }
        }
    }
}

// ------------------------------------------------------------------------------------
// grad_flux on triangles, physical mode, on the matrix cores (p <= 4: N_u, N_f <= 16).
//
// Every operator product of the element is a dense (16 x 16) x (16 x 16) product of the
// zero-padded operator with the values of 16 elements (one column per element): one wave
// takes 16 elements and applies each operator with four 16x16x4 MFMAs (K = 16 in four
// steps of 4), in the precision of the form (v_mfma_f64_16x16x4f64 / _f32_16x16x4f32).
// A field of the 16 elements lives in registers: lane l = 16 g + c holds, in register r,
// the value at row(g, r) of element c (row = point or flux-point index). The result rows
// of the instruction come out in that same order, so the product of one operator is the
// input of the next without any exchange between lanes, provided the operator's columns
// are fed in the matching order: in step s, lane (m, g) supplies entry (m, row(g, s)).
// row(g, r) = g + 4 r for the f64 instruction and 4 g + r for the f32 one (the result
// layouts of the two instructions). The wave runs the whole of Steps 1-5 and the volume
// part of Step 6 of its 16 elements without LDS or barriers; the pointwise work (fluxes,
// common fluxes) is done by each lane on the points it holds.
// ------------------------------------------------------------------------------------
template <typename R>
struct MfTile;
template <>
struct MfTile<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ static v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static constexpr int row(int g, int r) { return g + 4 * r; }
};
template <>
struct MfTile<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ static v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static constexpr int row(int g, int r) { return 4 * g + r; }
};

// tiles of 16 elements per wave; a grid-stride loop over tiles keeps the operators in
// registers across the wave's tiles
constexpr int TRI_MF_WAVES = 4;
constexpr int64_t TRI_MF_MAX_BLOCKS = 2048;

template <typename R, int P, bool NPHI>
__global__ __launch_bounds__(64 * TRI_MF_WAVES) void k_tri_grad_flux_mf(GFArgs<R> a) {
    using S = TriShape<P>;
    using T = MfTile<R>;
    using v4 = typename T::v4;
    using M = Math<R>;
    constexpr int NU = S::NU, NF = S::NF, G = S::G;
    constexpr int NV = NPHI ? 0 : 1;
    static_assert(NU <= 16 && NF <= 16, "one 16 x 16 tile per operator");
    const int lane = threadIdx.x & 63;
    const int c = lane & 15, g = lane >> 4;

    // A operands in LDS, lane (m, g) of step s holding Op[m][row(g, s)] (operator o at
    // s_op[o][s][lane]: conflict-free reads), and the per-lane constants of the rows a lane
    // holds (reference point coordinates, flux point coordinates and normals). Kept in LDS
    // and read where used, they leave the registers to the 16-element fields.
    enum { O_M0, O_D0, O_D1, O_L, O_DH0, O_DH1, NOP };
    enum { C_UR0, C_UR1, C_FR0, C_FR1, C_NH0, C_NH1 };
    __shared__ R s_op[NOP][4][64];
    __shared__ R s_cst[6][4][64];
    for (int t = threadIdx.x; t < NOP * 4 * 64; t += 64 * TRI_MF_WAVES) {
        const int o = t >> 8, st = (t >> 6) & 3, l = t & 63;
        const int m = l & 15, k = MfTile<R>::row(l >> 4, st);
        R val = R(0);
        if (o == O_M0) val = (m < NF && k < NU) ? a.ops[S::OM0 + m * NU + k] : R(0);
        else if (o == O_D0) val = (m < NU && k < NU) ? a.ops[S::OD0 + m * NU + k] : R(0);
        else if (o == O_D1) val = (m < NU && k < NU) ? a.ops[S::OD1 + m * NU + k] : R(0);
        else if (o == O_L) val = (m < NU && k < NF) ? a.ops[S::OL + m * NF + k] : R(0);
        else if (o == O_DH0) val = (m < NU && k < NU) ? a.ops[S::ODH0 + m * NU + k] : R(0);
        else val = (m < NU && k < NU) ? a.ops[S::ODH1 + m * NU + k] : R(0);
        s_op[o][st][l] = val;
    }
    for (int t = threadIdx.x; t < 4 * 64; t += 64 * TRI_MF_WAVES) {
        const int r = t >> 6, l = t & 63;
        const int j = MfTile<R>::row(l >> 4, r);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            s_cst[C_UR0 + i][r][l] = j < NU ? a.ops[S::OUR + 2 * j + i] : R(0);
            s_cst[C_FR0 + i][r][l] = j < NF ? a.ops[S::OFR + 2 * j + i] : R(0);
            s_cst[C_NH0 + i][r][l] = j < NF ? a.ops[S::ONH + 2 * j + i] : R(0);
        }
    }
    __syncthreads();
    auto apply = [&](int o, const v4& x, v4 acc) {
#pragma unroll
        for (int st = 0; st < 4; ++st) acc = T::mma(s_op[o][st][lane], x[st], acc);
        return acc;
    };
    auto cst = [&](int which, int r) { return s_cst[which][r][lane]; };

    const int64_t ntiles = (a.E + 15) / 16;
    const int64_t wstride = (int64_t)gridDim.x * TRI_MF_WAVES;
    for (int64_t tile = (int64_t)blockIdx.x * TRI_MF_WAVES + (threadIdx.x >> 6); tile < ntiles;
         tile += wstride) {
        // keeps the LDS reads of the operators and constants inside the loop
        asm volatile("" ::: "memory");
        const int64_t e = tile * 16 + c;
        const bool ev = e < a.E;
        const uint32_t ue = (uint32_t)(ev ? e : 0);
        // ---- loads: state, slot codes, partner traces, geometry ----------------------------
        v4 u[2];
        int code[4];
        R ptr[2][4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = T::row(g, r);
#pragma unroll
            for (int v = 0; v < 2; ++v) u[v][r] = (ev && j < NU) ? gld(a.u[v], ue * NU + j) : R(0);
            code[r] = (ev && j < NF) ? gld(a.nbr, ue * NF + j) : -2;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int v = 0; v < 2; ++v)
                ptr[v][r] = code[r] >= 0 ? gld(a.Tp[v], (uint32_t)(code[r] >> 1)) : R(0);
        R gg[G];
#pragma unroll
        for (int q = 0; q < G; ++q) gg[q] = ev ? gld(a.geo, ue * G + q) : (q == 10 ? R(1) : R(0));
        const R det = gg[10];
        const R* Ji = gg + 6;                       // Jinv[k][i] = Ji[k * 2 + i]

        // ---- Steps 1-3: own traces, LDG jumps, corrected gradient --------------------------
        const v4 z = {R(0), R(0), R(0), R(0)};
        v4 tf[2], q[2][2];
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            tf[v] = apply(O_M0, u[v], z);
            v4 qt[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                v4 jn;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    jn[r] = (code[r] >= 0 && (code[r] & 1)) ? cst(C_NH0 + k, r) * (ptr[v][r] - tf[v][r]) : R(0);
                qt[k] = apply(k == 0 ? O_D0 : O_D1, u[v], z);
                qt[k] = apply(O_L, jn, qt[k]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) q[v][i][r] = Ji[0 * 2 + i] * qt[0][r] + Ji[1 * 2 + i] * qt[1][r];
        }

        // ---- Step 5: common normal flux at the owned and boundary flux points ------------
        {
            v4 qf[2][2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                qf[0][i] = apply(O_M0, q[0][i], z);
                if constexpr (!NPHI) qf[1][i] = apply(O_M0, q[1][i], z);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (!(code[r] == -1 || (code[r] >= 0 && (code[r] & 1)))) continue;
                const R n0 = cst(C_NH0, r), n1 = cst(C_NH1, r);
                R nr[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) nr[i] = Ji[0 * 2 + i] * n0 + Ji[1 * 2 + i] * n1;
                const R rmag = M::rsqrt_(nr[0] * nr[0] + nr[1] * nr[1]);
                nr[0] *= rmag;
                nr[1] *= rmag;
                R x[2], vel[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) x[i] = gg[i] + gg[2 + i * 2 + 0] * cst(C_FR0, r) + gg[2 + i * 2 + 1] * cst(C_FR1, r);
                velocity<R, 2>(a.ph, x, vel);
                const R v2 = vel[0] * vel[0] + vel[1] * vel[1];
                const R vn = vel[0] * nr[0] + vel[1] * nr[1];
                const R mm = max_sqrt(v2, a.ph.gamma);
                const R qn0 = qf[0][0][r] * nr[0] + qf[0][1][r] * nr[1];
                const R qnn = qf[NV][0][r] * nr[0] + qf[NV][1][r] * nr[1];
                const R g2 = qf[NV][0][r] * qf[NV][0][r] + qf[NV][1][r] * qf[NV][1][r];
                const R rn = M::rsqrt_(g2 + a.ph.delta_n * a.ph.delta_n);
                const R pL = tf[0][r], sL = tf[1][r];
                const R pR = code[r] >= 0 ? ptr[0][r] : pL, sR = code[r] >= 0 ? ptr[1][r] : sL;
                const R fvn = mm * (a.ph.eps * qn0 - a.ph.gamma * pL * (R(1) - pL) * qnn * rn);
                const R F0 = R(0.5) * (pL + pR) * vn - fvn + a.ph.tau * (pL - pR);
                const R F1 = R(0.5) * (sL + sR) * vn + a.ph.tau * (sL - sR);
                const uint32_t slot = ue * NF + T::row(g, r);
                gst(a.Fp[0], slot, F0);
                gst(a.Fp[1], slot, F1);
            }
        }

        // ---- Step 4: transformed fluxes at the solution points -----------------------------
        v4 ft[2][2];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool pv = T::row(g, r) < NU;
            R x[2], vel[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) x[i] = gg[i] + gg[2 + i * 2 + 0] * cst(C_UR0, r) + gg[2 + i * 2 + 1] * cst(C_UR1, r);
            velocity<R, 2>(a.ph, x, vel);
            const R v2 = vel[0] * vel[0] + vel[1] * vel[1];
            const R g2 = q[NV][0][r] * q[NV][0][r] + q[NV][1][r] * q[NV][1][r];
            const R mm = max_sqrt(v2, a.ph.gamma);
            const R rn = M::rsqrt_(g2 + a.ph.delta_n * a.ph.delta_n);
            const R phi = u[0][r], psi = u[1][r];
            const R sharp = a.ph.gamma * phi * (R(1) - phi) * rn;
            R f0[2], f1[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const R fvis = mm * (a.ph.eps * q[0][i][r] - sharp * q[NV][i][r]);
                f0[i] = phi * vel[i] - fvis;
                f1[i] = psi * vel[i];
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                ft[0][k][r] = pv ? det * (Ji[k * 2 + 0] * f0[0] + Ji[k * 2 + 1] * f0[1]) : R(0);
                ft[1][k][r] = pv ? det * (Ji[k * 2 + 0] * f1[0] + Ji[k * 2 + 1] * f1[1]) : R(0);
            }
        }

        // ---- Step 6, volume part: P = D_0 f~_0 + D_1 f~_1 - Lift (nhat . M0 f~)
        // = DH_0 f~_0 + DH_1 f~_1, the lifting folded into DH_k = D_k - Lift diag(nhat_k) M0
        // (two products per variable instead of five) -----------------------------------
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            v4 pacc = apply(O_DH0, ft[v][0], z);
            pacc = apply(O_DH1, ft[v][1], pacc);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = T::row(g, r);
                if (ev && j < NU) gst(a.P[v], ue * NU + j, pacc[r]);
            }
        }
    }
}

// update on triangles: Step 6 face part and the RK4 combine, then the own traces of the next
// stage input (UP_RK), or the residual (UP_RESID).
template <typename R, int P, int V, int KIND>
__global__ __launch_bounds__(256) void k_tri_update(UPArgs<R> a) {
    using S = TriShape<P>;
    constexpr int NU = S::NU, NF = S::NF, EPB = S::EPB, G = S::G;
    constexpr int XU = EPB * NU, XF = EPB * NF;
    __shared__ R s_M0[NF * NU];
    __shared__ R s_L[NU * NF];
    __shared__ R s_F[V][XF];
    __shared__ R s_y[KIND == UP_RK ? V : 1][KIND == UP_RK ? XU : 1];

    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    const int nel = (int)((a.E - e0) < EPB ? (a.E - e0) : EPB);
    const bool pt = tid < nel * NU;
    const bool fp = tid < nel * NF;
    const int pe = tid / NU, pi = tid - pe * NU;
    const int fi = tid - (tid / NF) * NF;
    for (int i = tid; i < NF * NU; i += 256) {
        s_M0[i] = a.ops[S::OM0 + i];
        s_L[i] = a.ops[S::OL + i];
    }
    R rP[V], rU[V], rA[V], det = R(1);
    if (pt) {
        det = a.geo[(e0 + pe) * G + 2 + 8];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            rP[v] = a.P[v][e0 * NU + tid];
            if constexpr (KIND == UP_RK) {
                rU[v] = a.un[v][e0 * NU + tid];
                rA[v] = a.first ? R(0) : a.acc[v][e0 * NU + tid];
            }
        }
    }
    if (fp) {
        const int code = a.nbr[e0 * NF + tid];
        // the owner's (or, on a boundary, the own) common flux; minus the owner's otherwise;
        // transformed with this element's |J| |J^-T nhat|
        const bool mine = code < 0 || (code & 1);
        const R* gf = a.geo + (e0 + tid / NF) * G;
        const R n0 = a.ops[S::ONH + 2 * fi], n1 = a.ops[S::ONH + 2 * fi + 1];
        const R r0 = gf[6 + 0] * n0 + gf[6 + 2] * n1, r1 = gf[6 + 1] * n0 + gf[6 + 3] * n1;
        const R sc = gf[10] * Math<R>::sqrt_(r0 * r0 + r1 * r1);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const R f = a.Fp[v][mine ? e0 * NF + tid : (code >> 1)];
            s_F[v][tid] = mine ? sc * f : -(sc * f);
        }
    }
    __syncthreads();
    if (pt) {
        const R rdet = R(1) / det;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            R acc = rP[v];
            for (int f = 0; f < NF; ++f) acc += s_L[pi * NF + f] * s_F[v][pe * NF + f];
            const R res = -acc * rdet;
            if constexpr (KIND == UP_RESID) {
                a.res[v][e0 * NU + tid] = res;
            } else {
                using M = Math<R>;
                R nx;
                if (!a.last) {
                    a.acc[v][e0 * NU + tid] = M::fma_(a.bcoef, res, rA[v]);
                    nx = M::fma_(a.ccoef, res, rU[v]);
                    a.us[v][e0 * NU + tid] = nx;
                } else {
                    nx = M::fma_(a.ccoef, M::fma_(a.bcoef, res, rA[v]), rU[v]);
                    a.un[v][e0 * NU + tid] = nx;
                    if (a.uo[0]) a.uo[v][e0 * NU + tid] = nx;
                }
                s_y[v][tid] = nx;
                const R lim = (v == 0 && V == 2) ? R(10) : R(1e30);
                if (!(Math<R>::fabs_(nx) <= lim)) *a.flag = 1;
            }
        }
    }
    if constexpr (KIND == UP_RK) {
        __syncthreads();
        if (fp) {
            const int fe = tid / NF;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R acc = R(0);
                for (int i = 0; i < NU; ++i) acc += s_M0[fi * NU + i] * s_y[v][fe * NU + i];
                a.Tp[v][e0 * NF + tid] = acc;
            }
        }
    }
}

// own traces of a given state (after set_state / reset)
template <typename R, int P, int V>
__global__ __launch_bounds__(256) void k_tri_trace(TRArgs<R> a) {
    using S = TriShape<P>;
    constexpr int NU = S::NU, NF = S::NF, EPB = S::EPB;
    __shared__ R s_M0[NF * NU];
    __shared__ R s_y[V][EPB * NU];
    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    const int nel = (int)((a.E - e0) < EPB ? (a.E - e0) : EPB);
    for (int i = tid; i < NF * NU; i += 256) s_M0[i] = a.ops[S::OM0 + i];
#pragma unroll
    for (int v = 0; v < V; ++v)
        if (tid < nel * NU) s_y[v][tid] = a.u[v][e0 * NU + tid];
    __syncthreads();
    if (tid < nel * NF) {
        const int fe = tid / NF, fi = tid - fe * NF;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            R acc = R(0);
            for (int i = 0; i < NU; ++i) acc += s_M0[fi * NU + i] * s_y[v][fe * NU + i];
            a.Tp[v][e0 * NF + tid] = acc;
        }
    }
}

// FP64 quadrature reduction with the nodal weights W[i] of the element
template <typename R, int P>
__global__ __launch_bounds__(REDUCE_THREADS) void k_tri_reduce(RDArgs<R> a) {
    constexpr int NU = TriShape<P>::NU;
    __shared__ double s_w[REDUCE_THREADS / 64];
    const int64_t total = a.E * NU;
    double acc = 0.0;
    for (int64_t idx = (int64_t)blockIdx.x * REDUCE_THREADS + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * REDUCE_THREADS) {
        const int64_t e = idx / NU;
        const int i = (int)(idx - e * NU);
        double f = (double)a.field[idx];
        if (a.kind == 2) {
            const double df = f - (double)a.ref[idx];
            acc += df * df;
            continue;
        }
        if (a.kind == 1) f = ::fabs(f - (double)a.ref[idx]);
        acc += a.det64[e] * a.w64[i] * f;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s_w[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int i = 0; i < REDUCE_THREADS / 64; ++i) r += s_w[i];
        a.partial[blockIdx.x] = r;
    }
}

template <typename R, int P>
struct TriImpl {
    using S = TriShape<P>;
    static unsigned grid(int64_t E) { return (unsigned)((E + S::EPB - 1) / S::EPB); }
    template <int MODE, bool NPHI>
    static void gf(const GFArgs<R>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
        if constexpr (MODE == GF_PHYS && P <= 4) {
            const int64_t waves = (a.E + 15) / 16;
            const int64_t blocks = (waves + TRI_MF_WAVES - 1) / TRI_MF_WAVES;
            hipExtLaunchKernelGGL((k_tri_grad_flux_mf<R, P, NPHI>),
                                  dim3((unsigned)(blocks < TRI_MF_MAX_BLOCKS ? blocks : TRI_MF_MAX_BLOCKS)),
                                  dim3(64 * TRI_MF_WAVES), 0, st, e0, e1, 0, a);
        } else {
            hipExtLaunchKernelGGL((k_tri_grad_flux<R, P, MODE, NPHI>), dim3(grid(a.E)), dim3(256),
                                  0, st, e0, e1, 0, a);
        }
    }
    static void grad_flux(int mode, int nvar, const GFArgs<R>& a, hipStream_t st, hipEvent_t e0,
                          hipEvent_t e1) {
        (void)nvar;
        switch (mode) {
            case GF_PHYS:
                if (a.nphi) gf<GF_PHYS, true>(a, st, e0, e1);
                else gf<GF_PHYS, false>(a, st, e0, e1);
                break;
            case GF_PRECOND: gf<GF_PRECOND, false>(a, st, e0, e1); break;
            case GF_SIGN: gf<GF_SIGN, false>(a, st, e0, e1); break;
            default: gf<GF_SENSOR, false>(a, st, e0, e1); break;
        }
    }
    static void update(int kind, int nvar, const UPArgs<R>& a, hipStream_t st, hipEvent_t e0,
                       hipEvent_t e1) {
        const dim3 g(grid(a.E)), b(256);
        if (nvar == 2) {
            if (kind == UP_RK) hipExtLaunchKernelGGL((k_tri_update<R, P, 2, UP_RK>), g, b, 0, st, e0, e1, 0, a);
            else hipExtLaunchKernelGGL((k_tri_update<R, P, 2, UP_RESID>), g, b, 0, st, e0, e1, 0, a);
        } else {
            if (kind == UP_RK) hipExtLaunchKernelGGL((k_tri_update<R, P, 1, UP_RK>), g, b, 0, st, e0, e1, 0, a);
            else hipExtLaunchKernelGGL((k_tri_update<R, P, 1, UP_RESID>), g, b, 0, st, e0, e1, 0, a);
        }
    }
    static void trace(int nvar, const TRArgs<R>& a, hipStream_t st) {
        if (nvar == 2) hipLaunchKernelGGL((k_tri_trace<R, P, 2>), dim3(grid(a.E)), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_tri_trace<R, P, 1>), dim3(grid(a.E)), dim3(256), 0, st, a);
    }
    static void reduce(const RDArgs<R>& a, int nblocks, hipStream_t st) {
        hipLaunchKernelGGL((k_tri_reduce<R, P>), dim3(nblocks), dim3(REDUCE_THREADS), 0, st, a);
    }
};

template <typename R, int P>
bool tri_fill(Launchers<R>* L) {
    L->epb = TriShape<P>::EPB;
    L->nt = 256;
    L->ngeo = TriShape<P>::G;
    L->grad_flux = &TriImpl<R, P>::grad_flux;
    L->update = &TriImpl<R, P>::update;
    L->trace = &TriImpl<R, P>::trace;
    L->reduce = &TriImpl<R, P>::reduce;
    return true;
}

}  // namespace

template <typename R>
bool get_tri_launchers(int p, Launchers<R>* L) {
    switch (p) {
        case 1: return tri_fill<R, 1>(L);
        case 2: return tri_fill<R, 2>(L);
        case 3: return tri_fill<R, 3>(L);
        case 4: return tri_fill<R, 4>(L);
        case 5: return tri_fill<R, 5>(L);
        default: return false;
    }
}
template bool get_tri_launchers<double>(int, Launchers<double>*);
template bool get_tri_launchers<float>(int, Launchers<float>*);

}  // namespace pcpf
