// HIP kernels of the FR-PCPF residual for gfx950 (tensor-product quads/hexes):
// templates, instantiated per dimension and precision by pcpf_kernels_{2d,3d}_{f64,f32}.hip.
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
// viscous flux. Hence only two fields cross element boundaries per stage: the traces of
// - faces, pushed by update into the owner's + face slots Tp, and the common flux, which
// grad_flux writes once into its own + face slots Fp and which update reads, negated, for
// the neighbour's - face. Both face arrays are planar by reference direction, [D][E][NFA]:
// the NFA points of one face of consecutive elements are consecutive, so the block-sized
// runs of every face access (traces pushed to e - stride_k, fluxes gathered from there)
// are contiguous. Boundary faces (no neighbour) use the ghost state B(u) = u, B(q) = q of
// §3.3 and are computed by the element itself; a boundary - face flux goes to plane D + k
// of Fp.
#pragma once

#include <hip/hip_ext.h>

#include <cmath>
#include <type_traits>

#include "pcpf_device.h"
#include "pcpf_internal.h"
#include "pcpf_mfma.h"

namespace pcpf {
namespace {

using namespace dev;

// ------------------------------------------------------------------------------------
// grad_flux: Steps 1-5 for the elements of one block.
//   GF_PHYS     u = [phi, psi]: corrected gradients, fluxes at solution points, partial
//               divergence P = sum_k DH_k f~_k, common fluxes on owned faces.
//   GF_PRECOND  psi only: sensor nu_e, g = -nu_e grad psi, source S = sgn (1 - |q|),
//               P = sum_k DH_k g~_k - |J| S, common fluxes on owned faces.
//   GF_SIGN     psi0 only: smeared sign tanh(psi0 / max(|grad psi0|, delta_g)).
//   GF_SENSOR   psi only: the element viscosity nu_e.
// AXIS: every element is axis-aligned (diagonal J): the metric terms reduce to one
// product per component, face normals are +-e_k, and trigonometric velocity fields come
// from per-element tables of sin^2(pi x_k), sin(2 pi x_k) at the n nodes and both ends.
// Phases: A loads (state, operators, geometry, neighbour traces, face normals, velocity
// tables) | B corrected gradient q and fluxes f~ at solution points -> LDS | C common
// fluxes on owned face points -> global, and P = sum_k DH_k f~_k -> global.
// ------------------------------------------------------------------------------------
// Occupancy target (waves per SIMD) of the physical grad_flux kernel; 0 leaves the
// register budget to the compiler.
#ifndef PCPF_GF_WAVES
#define PCPF_GF_WAVES 0
#endif

// MF: the line operators of the gradient (DT, and lp for the own traces) and of the
// divergence (DH) run on the matrix cores with bf16 operands and fp32 accumulation (the
// BF16 form; R = float), each line taken as deviations from its mean with hi / lo bf16
// splits of operator and data (three MFMAs per product); the pointwise flux math, the face
// interpolations and the sensor stay in fp32 on the vector units.
// NPHI (physical mode): the interface normal of the sharpening flux comes from phi instead
// of psi, the unpreconditioned conservative phase field of §2.
template <typename R, int D, int P, int MODE, bool AXIS, bool MF = false, bool NPHI = false>
__global__ __launch_bounds__((Shape<D, P>::NT))
#if PCPF_GF_WAVES > 0
__attribute__((amdgpu_waves_per_eu(PCPF_GF_WAVES)))
#endif
void k_grad_flux(GFArgs<R> a) {
    static_assert(!MF || std::is_same<R, float>::value, "the matrix-core form is fp32");
    using S = Shape<D, P>;
    constexpr int N = S::N, NU = S::NU, NFA = S::NFA, EPB = S::EPB, NT = S::NT, G = S::GEO;
    constexpr int V = (MODE == GF_PHYS) ? 2 : 1;
    constexpr int NV = NPHI ? 0 : V - 1;                // variable the interface normal is of
    constexpr int NOPS = ops_size(N);
    constexpr bool FLUX = (MODE == GF_PHYS || MODE == GF_PRECOND);
    constexpr bool SENS = (MODE == GF_PRECOND || MODE == GF_SENSOR);
    constexpr bool GRAD = (MODE != GF_SENSOR);
    constexpr bool TAB = (MODE == GF_PHYS) && AXIS;      // velocity tables possible
    constexpr int NPF = D * NFA;                         // points on the + faces of one element
    constexpr int NTB = N + 2;                           // table positions per axis
    constexpr int XST = EPB * NU;                        // stride of one field in s_x / s_f
    constexpr int NX = (V * D > 2 ? V * D : 2) * XST;
    using M = Math<R>;

    __shared__ R s_ops[NOPS];
    __shared__ R s_geo[EPB * G];
    __shared__ R s_u[V][EPB * NU];
    __shared__ R s_x[NX];                                // q (or sensor scratch)
    __shared__ R s_f[FLUX ? V * D * XST : 1];            // f~ at solution points
    __shared__ R s_nb[GRAD ? V : 1][GRAD ? EPB * NPF : 1];  // + face neighbour traces
    __shared__ R s_vt[TAB ? EPB * D * NTB * 2 : 1];
    __shared__ R s_nu[EPB];
    __shared__ R s_fn[FLUX && !AXIS ? EPB * D * (D + 1) : 1];  // + face unit normal, scale
    __shared__ int s_nbr[EPB * 2 * D];
    __shared__ R s_tr[MF ? V * D * EPB * NFA : 1];       // own + face traces (MF)

    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)block_chunk<R>(a.E * NU) * EPB;
    const int nel = (int)((a.E - e0) < EPB ? (a.E - e0) : EPB);
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
    const bool trig = a.ph.vel_kind == PCPF_VEL_SINGLE_VORTEX || a.ph.vel_kind == PCPF_VEL_LEVEQUE3D;

    // ---- A: loads. Every global load of the phase is issued into registers before the
    // first wait, then the values go to LDS. All loads are indexed by this block's own
    // elements: the neighbours pushed their traces into this element's + face slots.
    constexpr int I_OPS = (NOPS + NT - 1) / NT;
    constexpr int I_GEO = (EPB * G + NT - 1) / NT;
    constexpr int I_NBR = (EPB * 2 * D + NT - 1) / NT;
    constexpr int I_U = (EPB * NU + NT - 1) / NT;
    constexpr int I_NB = (EPB * NPF + NT - 1) / NT;
    constexpr int I_TB = TAB ? (EPB * D * NTB * 2 + NT - 1) / NT : 1;
    R r_ops[I_OPS], r_geo[I_GEO], r_u[V][I_U];
    int32_t r_nbr[I_NBR];
#pragma unroll
    for (int j = 0; j < I_OPS; ++j) {
        const int i = tid + j * NT;
        r_ops[j] = gld_in(a.ops, i, NOPS);
    }
#pragma unroll
    for (int j = 0; j < I_GEO; ++j) {
        const int i = tid + j * NT;
        r_geo[j] = gld_in(a.geo + e0 * G, i, nel * G);
    }
#pragma unroll
    for (int j = 0; j < I_NBR; ++j) {
        const int i = tid + j * NT;
        r_nbr[j] = gld_in(a.nbr + e0 * 2 * D, i, nel * 2 * D);
    }
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
        for (int j = 0; j < I_U; ++j) {
            const int i = tid + j * NT;
            r_u[v][j] = gld_in(a.u[v] + e0 * NU, i, nel * NU);
        }
    // + face normal inputs (row k of J^-1 and |J|) of this thread's (element, face)
    R r_ji[FLUX ? D : 1], r_det = R(1);
    const bool fn_thread = FLUX && !AXIS && tid < nel * D;
    if constexpr (FLUX) {
        if (fn_thread) {
            const int el = tid / D, k = tid - el * D;
            const R* gb = a.geo + e0 * G;
#pragma unroll
            for (int i = 0; i < D; ++i) r_ji[i] = gld(gb, el * G + D + D * D + k * D + i);
            r_det = gld(gb, el * G + D + 2 * D * D);
        }
    }
    // neighbour traces on the + faces, pushed here by the neighbours (boundary + face
    // slots are zeroed when the context is created and never written)
    // slots: lanes run over [k][el NFA + t], contiguous within each direction's plane
    constexpr int KSEG = S::KSEG;
    const uint32_t Eu = (uint32_t)a.E;
    R r_nb[GRAD ? I_NB : 1][V];
    int nb_pos[GRAD ? I_NB : 1];
    if constexpr (GRAD) {
#pragma unroll
        for (int j = 0; j < I_NB; ++j) {
            const int it = tid + j * NT;
            int k = it / KSEG;
            int r = it - k * KSEG;
            const bool ok = k < D && r < nel * NFA;
            nb_pos[j] = ok ? (r / NFA) * NPF + k * NFA + (r % NFA) : -1;
            k = k < D ? k : D - 1;
            r = r < nel * NFA ? r : nel * NFA - 1;
            const uint32_t gi = ((uint32_t)k * Eu + (uint32_t)e0) * NFA + (uint32_t)r;
#pragma unroll
            for (int v = 0; v < V; ++v) r_nb[j][v] = gld(a.Tp[v], gi);
        }
    }
    // velocity tables of the block's elements (sin^2(pi x_k) and sin(2 pi x_k) at the line
    // positions of every axis; stored with the geometry, they depend on the mesh only)
    R r_vt[I_TB];
    if constexpr (TAB) {
#pragma unroll
        for (int j = 0; j < I_TB; ++j) {
            const int it = tid + j * NT;
            r_vt[j] = trig ? gld_in(a.vtab + e0 * D * NTB * 2, it, nel * D * NTB * 2) : R(0);
        }
    }
    // registers -> LDS
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
    if constexpr (GRAD) {
#pragma unroll
        for (int j = 0; j < I_NB; ++j)
            if (nb_pos[j] >= 0)
#pragma unroll
                for (int v = 0; v < V; ++v) s_nb[v][nb_pos[j]] = r_nb[j][v];
    }
    // outward unit normal n = J^-T e_k / |J^-T e_k| and scale |J| |J^-T e_k| of face +k
    if constexpr (FLUX && !AXIS) {
        if (fn_thread) {
            R mag2 = R(0);
#pragma unroll
            for (int i = 0; i < D; ++i) mag2 += r_ji[i] * r_ji[i];
            const R mag = M::sqrt_(mag2);
            R* fn = &s_fn[tid * (D + 1)];
#pragma unroll
            for (int i = 0; i < D; ++i) fn[i] = r_ji[i] / mag;
            fn[D] = r_det * mag;
        }
    }
    if constexpr (TAB) {
        if (trig) {
#pragma unroll
            for (int j = 0; j < I_TB; ++j)
                if (tid + j * NT < nel * D * NTB * 2) s_vt[tid + j * NT] = r_vt[j];
        }
    }
    __syncthreads();

    // ---- sensor (§3.2): modal coefficients by one 1D transform per direction -----------
    if constexpr (SENS) {
        const R* VI = &s_ops[op_vinv(N)];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const R* src = (k == 0) ? s_u[0] : s_x + ((k - 1) & 1) * XST;
            R* dst = s_x + (k & 1) * XST;
            if (pt) {
                R acc = R(0);
                const int b0 = le * NU + ip - mi[k] * st<N>(k);
#pragma unroll
                for (int q = 0; q < N; ++q) acc += VI[mi[k] * N + q] * src[b0 + q * st<N>(k)];
                dst[tid] = acc;
            }
            __syncthreads();
        }
        const R* chi = s_x + ((D - 1) & 1) * XST;
        // modal energies of each element. Small elements: one thread per element sums its
        // points in order; large elements (N_u >= 64): a wave per element, lanes over its
        // points, then a fixed butterfly (lane 0's sum is used: deterministic).
        auto energies = [&](int el, int i0, int di, R& ea, R& et) {
            for (int i = i0; i < NU; i += di) {
                const R c = chi[el * NU + i];
                ea += c * c;
                int r = i, top = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    top |= ((r % N) == P);
                    r /= N;
                }
                if (top) et += c * c;
            }
        };
        auto set_nu = [&](int el, R ea, R et) {
            const R nu = visc_ramp(ea, et, a.ph.s0, a.ph.kappa, a.ph.nu_max);
            s_nu[el] = nu;
            if constexpr (MODE == GF_SENSOR) gst(a.out + e0, el, nu);
        };
        if constexpr (NU < 64) {
            if (tid < nel) {
                R ea = R(0), et = R(0);
                energies(tid, 0, 1, ea, et);
                set_nu(tid, ea, et);
            }
        } else {
            const int swave = __builtin_amdgcn_readfirstlane(tid >> 6);
            const int slane = tid & 63;
            for (int el = swave; el < nel; el += S::NW) {
                R ea = R(0), et = R(0);
                energies(el, slane, 64, ea, et);
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    ea += __shfl_xor(ea, off, 64);
                    et += __shfl_xor(et, off, 64);
                }
                if (slane == 0) set_nu(el, ea, et);
            }
        }
        __syncthreads();
        if constexpr (MODE == GF_SENSOR) return;
    }

    if constexpr (GRAD) {
        // ---- B: corrected gradient (Steps 1-3) and fluxes at solution points (Step 4) ---
        // The matrix-core form first applies [DT; lp] along the lines of every direction
        // (16 lines per instruction): s_x <- DT u, s_tr <- the own + face trace lp u.
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int lane = tid & 63;
        // every lane of a wave takes part: unit j of the wave is direction k = u / WK,
        // lines (u % WK) * 64 + 16 g + lane % 16, g = 0..3 (wave-uniform k)
        auto mf_lines = [&](auto body) {
#pragma unroll
            for (int j = 0; j < S::UPW; ++j) {
                const int u = wave + j * S::NW;
                if (u >= S::NUNITS) break;
                const int k = u / S::WK;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int item = (u - k * S::WK) * 64 + 16 * g + (lane & 15);
                    const bool ok = item < nel * NFA;
                    const int el = ok ? item / NFA : 0, t = ok ? item - el * NFA : 0;
                    if (k == 0) {
                        body(std::integral_constant<int, 0>{}, ok, el, t, item);
                    } else if (k == 1) {
                        body(std::integral_constant<int, 1>{}, ok, el, t, item);
                    } else if constexpr (D == 3) {
                        body(std::integral_constant<int, 2>{}, ok, el, t, item);
                    }
                }
            }
        };
        if constexpr (MF) {
            const RowsSplit aG = mfma_rows_split<N + 1, N>(
                [&](int i, int k) { return i < N ? s_ops[op_dt(N) + i * N + k] : s_ops[op_lp(N) + k]; },
                lane);
            mf_lines([&](auto KC, bool ok, int el, int t, int item) {
                constexpr int K = decltype(KC)::value;
                constexpr int SK = st<N>(K);
                const int base = el * NU + face_base<D, N>(K, t);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const f32x4 r = mfma_lines_split<N>(aG, s_u[v], ok, base, SK, lane);
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int row = 4 * (lane >> 4) + jj;
                        if (ok && row < N) s_x[(v * D + K) * XST + base + row * SK] = r[jj];
                        if (ok && row == N) s_tr[(v * D + K) * EPB * NFA + item] = r[jj];
                    }
                }
            });
            __syncthreads();
        }
        R Sdet = R(0);
        if (pt) {
            const R* gg = &s_geo[le * G];
            const R det = gg[D + 2 * D * D];
            const R* Ji = gg + D + D * D;            // Jinv[k][i] = Ji[k*D + i]
            const R* cp = &s_ops[op_cp(N)];
            R q[V][D];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R qt[D];
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    // + face with a neighbour: the LDG jump (nb - own trace) is lifted; the
                    // own-trace part is folded into DT = D1 - cp (x) lp
                    const bool hk = s_nbr[le * 2 * D + 2 * k + 1] >= 0;
                    const int tk = tang_index<D, N>(k, mi);
                    if constexpr (MF) {
                        // DT u from the matrix cores; on a boundary + face the "neighbour"
                        // trace is the own trace (no jump)
                        const R nbk = hk ? s_nb[v][le * NPF + k * NFA + tk]
                                         : s_tr[(v * D + k) * EPB * NFA + le * NFA + tk];
                        qt[k] = s_x[(v * D + k) * XST + tid] + cp[mi[k]] * nbk;
                    } else {
                        const R* Dk = &s_ops[hk ? op_dt(N) : OP_D1] + mi[k] * N;
                        const int b0 = le * NU + ip - mi[k] * st<N>(k);
                        R acc = R(0);
#pragma unroll
                        for (int b = 0; b < N; ++b) acc += Dk[b] * s_u[v][b0 + b * st<N>(k)];
                        // boundary + faces: s_nb holds 0 (those slots are never written)
                        acc += cp[mi[k]] * s_nb[v][le * NPF + k * NFA + tk];
                        qt[k] = acc;
                    }
                }
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    R acc;
                    if constexpr (AXIS) {
                        acc = Ji[i * D + i] * qt[i];
                    } else {
                        acc = R(0);
#pragma unroll
                        for (int k = 0; k < D; ++k) acc += Ji[k * D + i] * qt[k];
                    }
                    q[v][i] = acc;
                    s_x[(v * D + i) * XST + tid] = acc;
                }
            }
            if constexpr (MODE == GF_SIGN) {
                R g2 = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) g2 += q[0][i] * q[0][i];
                R g = M::sqrt_(g2);
                if (!(g > a.ph.delta_g)) g = a.ph.delta_g;
                gst(a.out + e0 * NU, tid, M::tanh_(s_u[0][tid] / g));
            }
            if constexpr (MODE == GF_PHYS) {
                const R* xi = &s_ops[op_xi(N)];
                R vel[D];
                if constexpr (TAB) {
                    if (trig) {
                        velocity_tab<R, D, NTB>(a.ph, &s_vt[le * D * NTB * 2], mi, vel);
                    } else {
                        R x[D];
#pragma unroll
                        for (int i = 0; i < D; ++i) x[i] = gg[i] + gg[D + i * D + i] * (xi[mi[i]] + R(1));
                        velocity_lin<R, D>(a.ph, x, vel);
                    }
                } else {
                    R x[D];
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        R acc = gg[i];
#pragma unroll
                        for (int j = 0; j < D; ++j) acc += gg[D + i * D + j] * (xi[mi[j]] + R(1));
                        x[i] = acc;
                    }
                    velocity<R, D>(a.ph, x, vel);
                }
                R v2 = R(0), g2 = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    v2 += vel[i] * vel[i];
                    g2 += q[NV][i] * q[NV][i];
                }
                const R mm = max_sqrt(v2, a.ph.gamma);
                const R rn = M::rsqrt_(g2 + a.ph.delta_n * a.ph.delta_n);
                const R phi = s_u[0][tid], psi = s_u[1][tid];
                const R sharp = a.ph.gamma * phi * (R(1) - phi) * rn;
                R f0[D], f1[D];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const R fvis = mm * (a.ph.eps * q[0][i] - sharp * q[NV][i]);
                    f0[i] = phi * vel[i] - fvis;
                    f1[i] = psi * vel[i];
                }
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    R a0, a1;
                    if constexpr (AXIS) {
                        a0 = Ji[k * D + k] * f0[k];
                        a1 = Ji[k * D + k] * f1[k];
                    } else {
                        a0 = R(0);
                        a1 = R(0);
#pragma unroll
                        for (int i = 0; i < D; ++i) {
                            a0 += Ji[k * D + i] * f0[i];
                            a1 += Ji[k * D + i] * f1[i];
                        }
                    }
                    s_f[(0 * D + k) * XST + tid] = det * a0;
                    s_f[((V - 1) * D + k) * XST + tid] = det * a1;
                }
            }
            if constexpr (MODE == GF_PRECOND) {
                const R nu = s_nu[le];
                R g2 = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) g2 += q[0][i] * q[0][i];
                const R g = M::sqrt_(g2);
                R sg = gld(a.sgn + e0 * NU, tid);
                if (a.sgn_current) {
                    // the printed smeared sign: psi0 over the current |grad psi|
                    R gd = g;
                    if (!(gd > a.ph.delta_g)) gd = a.ph.delta_g;
                    sg = M::tanh_(sg / gd);
                }
                Sdet = det * sg * (R(1) - g);
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    R acc;
                    if constexpr (AXIS) {
                        acc = Ji[k * D + k] * q[0][k];
                    } else {
                        acc = R(0);
#pragma unroll
                        for (int i = 0; i < D; ++i) acc += Ji[k * D + i] * q[0][i];
                    }
                    s_f[k * XST + tid] = -det * nu * acc;
                }
            }
        }
        if constexpr (MODE == GF_SIGN) return;
        __syncthreads();

        // ---- C: common normal fluxes on owned face points (Step 5) ----------------------
        // One face point per lane; each wave takes the points of one reference direction
        // K (compile-time in the body below). + faces are owned; - faces are computed here
        // only on boundaries (ghost state = interior state).
        auto face = [&](auto KC, auto SC, int el, int t, int32_t en) {
            constexpr int K = decltype(KC)::value;
            constexpr int SD = decltype(SC)::value;      // 1: + face, 0: - face
            constexpr int SK = st<N>(K);
            const int base = el * NU + face_base<D, N>(K, t);
            const R* l = &s_ops[SD ? op_lp(N) : op_lm(N)];
            const R* gg = &s_geo[el * G];
            R nrm[D], sc;
            if constexpr (AXIS) {
                // diagonal J: the unit normal of face +K is sign(Jinv_KK) e_K
                const R jk = gg[D + D * D + K * D + K];
                sc = gg[D + 2 * D * D] * M::fabs_(jk);
#pragma unroll
                for (int i = 0; i < D; ++i) nrm[i] = R(0);
                nrm[K] = ((jk > R(0)) == (SD == 1)) ? R(1) : R(-1);
            } else {
                const R* fn = &s_fn[(el * D + K) * (D + 1)];
                sc = fn[D];
#pragma unroll
                for (int i = 0; i < D; ++i) nrm[i] = SD ? fn[i] : -fn[i];
            }
            R uL[V], uR[V], qn[V], g2 = R(0);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R acc = R(0);
#pragma unroll
                for (int q = 0; q < N; ++q) acc += l[q] * s_u[v][base + q * SK];
                uL[v] = acc;
                uR[v] = (en >= 0) ? s_nb[v][el * NPF + K * NFA + t] : acc;
                // the normal component; in the physical mode all components of the variable
                // the interface normal is of (they enter its |grad|)
                R acc_n = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const bool need = !AXIS || (MODE == GF_PHYS && v == NV) || i == K;
                    if (!need) continue;
                    R qa = R(0);
#pragma unroll
                    for (int q = 0; q < N; ++q) qa += l[q] * s_x[(v * D + i) * XST + base + q * SK];
                    if constexpr (AXIS) {
                        if (i == K) acc_n = qa * nrm[K];
                    } else {
                        acc_n += qa * nrm[i];
                    }
                    if (MODE == GF_PHYS && v == NV) g2 += qa * qa;
                }
                qn[v] = acc_n;
            }
            // slot of this face point in plane K (+ face) or D + K (boundary - face)
            const uint32_t fo = (((uint32_t)(SD ? K : D + K)) * Eu + (uint32_t)(e0 + el)) * NFA + t;
            if constexpr (MODE == GF_PHYS) {
                const R* xi = &s_ops[op_xi(N)];
                R vel[D];
                int pos[D];
                {
                    int tt = t;
#pragma unroll
                    for (int m = 0; m < D; ++m) {
                        if (m == K) {
                            pos[m] = N + SD;
                        } else {
                            pos[m] = tt % N;
                            tt /= N;
                        }
                    }
                }
                if constexpr (TAB) {
                    if (trig) {
                        velocity_tab<R, D, NTB>(a.ph, &s_vt[el * D * NTB * 2], pos, vel);
                    } else {
                        R x[D];
#pragma unroll
                        for (int m = 0; m < D; ++m) {
                            const R xr = (m == K) ? (SD ? R(2) : R(0)) : xi[pos[m]] + R(1);
                            x[m] = gg[m] + gg[D + m * D + m] * xr;
                        }
                        velocity_lin<R, D>(a.ph, x, vel);
                    }
                } else {
                    R x[D];
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        R acc = gg[i];
#pragma unroll
                        for (int m = 0; m < D; ++m) {
                            const R xr = (m == K) ? (SD ? R(2) : R(0)) : xi[pos[m]] + R(1);
                            acc += gg[D + i * D + m] * xr;
                        }
                        x[i] = acc;
                    }
                    velocity<R, D>(a.ph, x, vel);
                }
                R v2 = R(0), vn = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    v2 += vel[i] * vel[i];
                    if constexpr (AXIS) {
                        if (i == K) vn = vel[K] * nrm[K];
                    } else {
                        vn += vel[i] * nrm[i];
                    }
                }
                const R mm = max_sqrt(v2, a.ph.gamma);
                const R rn = M::rsqrt_(g2 + a.ph.delta_n * a.ph.delta_n);
                const R pL = uL[0], pR = uR[0], sL = uL[1], sR = uR[1];
                const R fvn = mm * (a.ph.eps * qn[0] - a.ph.gamma * pL * (R(1) - pL) * qn[NV] * rn);
                const R F0 = R(0.5) * (pL + pR) * vn - fvn + a.ph.tau * (pL - pR);
                const R F1 = R(0.5) * (sL + sR) * vn + a.ph.tau * (sL - sR);
                const R G0 = sc * F0, G1 = sc * F1;
                gst(a.Fp[0], fo, G0);
                gst(a.Fp[1], fo, G1);
            } else {
                const R F = -s_nu[el] * qn[0] + a.ph.tau * (uL[0] - uR[0]);
                gst(a.Fp[0], fo, sc * F);
            }
        };
        // wave-uniform direction: each unit is one wave's worth of one direction's points
        auto face_pass = [&](auto SC) {
            constexpr int SD = decltype(SC)::value;
#pragma unroll
            for (int j = 0; j < S::UPW; ++j) {
                const int u = wave + j * S::NW;
                if (u >= S::NUNITS) break;
                const int k = u / S::WK;
                const int item = (u - k * S::WK) * 64 + lane;
                if (item >= nel * NFA) continue;
                const int el = item / NFA, t = item - el * NFA;
                const int32_t en = s_nbr[el * 2 * D + 2 * k + SD];
                if (SD == 0 && en >= 0) continue;
                if (k == 0) {
                    face(std::integral_constant<int, 0>{}, SC, el, t, en);
                } else if (k == 1) {
                    face(std::integral_constant<int, 1>{}, SC, el, t, en);
                } else if constexpr (D == 3) {
                    face(std::integral_constant<int, 2>{}, SC, el, t, en);
                }
            }
        };
        face_pass(std::integral_constant<int, 1>{});
        // - faces on a boundary (face 2k without a neighbour) exist only on meshes with
        // walls; the pass skips every point whose face has a neighbour
        if (a.bnd_minus) face_pass(std::integral_constant<int, 0>{});

        // ---- E: volume part of Step 6, P = sum_k DH_k f~_k (- |J| S) ---------------------
        if constexpr (MF) {
            // DH along the lines of every direction on the matrix cores, in place (the
            // direction-K field of s_f is touched only by the direction-K lines), then the
            // directions summed per point
            const RowsSplit aH = mfma_rows_split<N, N>(
                [&](int i, int k) { return s_ops[op_dh(N) + i * N + k]; }, lane);
            mf_lines([&](auto KC, bool ok, int el, int t, int item) {
                (void)item;
                constexpr int K = decltype(KC)::value;
                constexpr int SK = st<N>(K);
                const int base = el * NU + face_base<D, N>(K, t);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    R* fk = &s_f[(v * D + K) * XST];
                    const f32x4 r = mfma_lines_split<N>(aH, fk, ok, base, SK, lane);
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int row = 4 * (lane >> 4) + jj;
                        if (ok && row < N) fk[base + row * SK] = r[jj];
                    }
                }
            });
            __syncthreads();
            if (pt) {
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    R acc = R(0);
#pragma unroll
                    for (int k = 0; k < D; ++k) acc += s_f[(v * D + k) * XST + tid];
                    if constexpr (MODE == GF_PRECOND) acc -= Sdet;
                    gst(a.P[v] + e0 * NU, tid, acc);
                }
            }
        } else {
            // volume divergence of block point t (thread-point numbering)
            auto e_point = [&](int t) {
                const int l = t / NU, q = t - l * NU;
                int m[D];
                {
                    int r = q;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        m[k] = r % N;
                        r /= N;
                    }
                }
                const R* DH = &s_ops[op_dh(N)];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    R acc = R(0);
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const int b0 = l * NU + q - m[k] * st<N>(k);
#pragma unroll
                        for (int b = 0; b < N; ++b)
                            acc += DH[m[k] * N + b] * s_f[(v * D + k) * XST + b0 + b * st<N>(k)];
                    }
                    if constexpr (MODE == GF_PRECOND) acc -= Sdet;
                    gst(a.P[v] + e0 * NU, t, acc);
                }
            };
            // Physical mode with at most half of the waves carrying face units: the waves
            // without one also take the divergence of the points of a wave with one, so
            // that the face work and the divergence are spread over all the block's waves.
            constexpr bool SHARE = MODE == GF_PHYS && 2 * S::NUNITS <= S::NW;
            if constexpr (SHARE) {
                if (wave >= S::NUNITS) {
                    if (pt) e_point(tid);
                    if (wave < 2 * S::NUNITS) {
                        const int t2 = tid - 64 * S::NUNITS;
                        if (t2 < nel * NU) e_point(t2);
                    }
                }
            } else if (pt) {
                e_point(tid);
            }
        }
    }
}

// ------------------------------------------------------------------------------------
// grad_flux, physical mode, by element lines (3D, and 2D in FP32): the same Steps 1-5 and
// volume part of Step 6 as k_grad_flux, with every line product done in registers by one
// thread per element line instead of one LDS read per operator entry per point.
//   A   loads, as k_grad_flux.
//   B1  line threads (direction K uniform in a wave): the line's N values of each variable
//       from LDS, the corrected derivative along K at its N points (Step 3) to LDS, and in
//       registers the + face values of the line: the own trace, the neighbour's trace and
//       the interpolated K component of the gradient.
//   B2  line threads: the common flux of the + face point (Step 5), reading only the other
//       gradient components at the face; all threads: the flux at their solution points
//       (Step 4) to LDS (one point per thread, or a loop over the block's points where the
//       block has a wave per unit of line work only: 3D in FP32, lines_nt).
//   E1  line threads: DH_K applied along the line (volume part of Step 6) plus the lifting
//       of the line's + face common flux from B2, to LDS.
//   E2  all threads: P = the sum over the directions (fixed order), to global; the update
//       adds the lifting of the - face fluxes.
// On axis-aligned meshes the LDS holds the physical gradient (one metric factor per
// component); otherwise the reference components, transformed where they are used.
// ------------------------------------------------------------------------------------
// Occupancy target (waves per SIMD). In float64 the kernel holds 86-114 VGPRs, which caps
// it at 4-5 waves; forcing more, with a few registers spilled to scratch, overlaps the
// blocks' load, LDS and arithmetic phases better (96^3 p4: 2382 us at 4, 2141 at 5, 2066 at
// 6; 64^3 p3: 281 at 5, 268 at 6, 257 at 7). The float32 form fits 8 waves anyway.
constexpr int lines_waves(int p) { return p <= 3 ? 7 : 6; }
// STREAM: the state planes exceed the caches; the state loads and the P stores (each value
// read or written once per launch) go with the non-temporal hint.
template <typename R, int D, int P, bool AXIS, bool NPHI, bool STREAM>
__global__ __launch_bounds__((lines_nt<R, D, P>()))
__attribute__((amdgpu_waves_per_eu(lines_waves(P))))
void k_grad_flux_lines(GFArgs<R> a) {
    using S = Shape<D, P, 256, lines_nt<R, D, P>()>;
    constexpr int N = S::N, NU = S::NU, NFA = S::NFA, EPB = S::EPB, NT = S::NT, G = S::GEO;
    constexpr int V = 2;
    constexpr int NV = NPHI ? 0 : 1;               // variable the interface normal is of
    constexpr int NOPS = ops_size(N);
    constexpr int NPF = D * NFA;
    constexpr int NTB = N + 2;
    constexpr int XST = EPB * NU;
    constexpr int KSEG = S::KSEG;
    constexpr int UPW = S::UPW;
    using M = Math<R>;

    __shared__ R s_ops[NOPS];
    __shared__ R s_geo[EPB * G];
    __shared__ R s_u[V][XST];
    // one field of V D components per point, reused in place: the gradient (B1), the flux
    // at the point (B2, each thread overwriting its own point), the directions' DH f~ (E1,
    // each line thread overwriting its own line)
    __shared__ R s_x[V * D * XST];
    __shared__ R s_nb[V][EPB * NPF];                // + face neighbour traces
    __shared__ R s_vt[AXIS ? EPB * D * NTB * 2 : 1];
    __shared__ R s_fn[AXIS ? 1 : EPB * D * (D + 1)]; // + face unit normal, scale
    __shared__ int s_nbr[EPB * 2 * D];

    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)block_chunk<R>(a.E * NU) * EPB;
    const int nel = (int)((a.E - e0) < EPB ? (a.E - e0) : EPB);
    const uint32_t Eu = (uint32_t)a.E;
    const bool trig = a.ph.vel_kind == PCPF_VEL_SINGLE_VORTEX || a.ph.vel_kind == PCPF_VEL_LEVEQUE3D;

    // ---- A: loads (every global load issued before the first wait) ----------------------
    constexpr int I_OPS = (NOPS + NT - 1) / NT;
    constexpr int I_GEO = (EPB * G + NT - 1) / NT;
    constexpr int I_NBR = (EPB * 2 * D + NT - 1) / NT;
    constexpr int I_U = (EPB * NU + NT - 1) / NT;
    constexpr int I_NB = (EPB * NPF + NT - 1) / NT;
    constexpr int I_TB = AXIS ? (EPB * D * NTB * 2 + NT - 1) / NT : 1;
    R r_ops[I_OPS], r_geo[I_GEO], r_u[V][I_U];
    int32_t r_nbr[I_NBR];
#pragma unroll
    for (int j = 0; j < I_OPS; ++j) r_ops[j] = gld_in(a.ops, tid + j * NT, NOPS);
#pragma unroll
    for (int j = 0; j < I_GEO; ++j) r_geo[j] = gld_in(a.geo + e0 * G, tid + j * NT, nel * G);
#pragma unroll
    for (int j = 0; j < I_NBR; ++j) r_nbr[j] = gld_in(a.nbr + e0 * 2 * D, tid + j * NT, nel * 2 * D);
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
        for (int j = 0; j < I_U; ++j) {
            const int i = tid + j * NT;
            r_u[v][j] = gld_s<STREAM>(a.u[v] + e0 * NU, (uint32_t)(i < nel * NU ? i : nel * NU - 1));
        }
    R r_ji[D], r_det = R(1);
    const bool fn_thread = !AXIS && tid < nel * D;
    if constexpr (!AXIS) {
        if (fn_thread) {
            const int el = tid / D, k = tid - el * D;
            const R* gb = a.geo + e0 * G;
#pragma unroll
            for (int i = 0; i < D; ++i) r_ji[i] = gld(gb, el * G + D + D * D + k * D + i);
            r_det = gld(gb, el * G + D + 2 * D * D);
        }
    }
    // neighbour traces: lanes over [k][el NFA + t], contiguous in each direction's plane
    R r_nb[I_NB][V];
    int nb_pos[I_NB];
#pragma unroll
    for (int j = 0; j < I_NB; ++j) {
        const int it = tid + j * NT;
        int k = it / KSEG;
        int r = it - k * KSEG;
        const bool ok = k < D && r < nel * NFA;
        nb_pos[j] = ok ? (r / NFA) * NPF + k * NFA + (r % NFA) : -1;
        k = k < D ? k : D - 1;
        r = r < nel * NFA ? r : nel * NFA - 1;
        const uint32_t gi = ((uint32_t)k * Eu + (uint32_t)e0) * NFA + (uint32_t)r;
#pragma unroll
        for (int v = 0; v < V; ++v) r_nb[j][v] = gld(a.Tp[v], gi);
    }
    R r_vt[I_TB];
    if constexpr (AXIS) {
#pragma unroll
        for (int j = 0; j < I_TB; ++j)
            r_vt[j] = trig ? gld_in(a.vtab + e0 * D * NTB * 2, tid + j * NT, nel * D * NTB * 2) : R(0);
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
        if (nb_pos[j] >= 0)
#pragma unroll
            for (int v = 0; v < V; ++v) s_nb[v][nb_pos[j]] = r_nb[j][v];
    if constexpr (!AXIS) {
        if (fn_thread) {
            R mag2 = R(0);
#pragma unroll
            for (int i = 0; i < D; ++i) mag2 += r_ji[i] * r_ji[i];
            const R mag = M::sqrt_(mag2);
            R* fn = &s_fn[tid * (D + 1)];
#pragma unroll
            for (int i = 0; i < D; ++i) fn[i] = r_ji[i] / mag;
            fn[D] = r_det * mag;
        }
    }
    if constexpr (AXIS) {
        if (trig) {
#pragma unroll
            for (int j = 0; j < I_TB; ++j)
                if (tid + j * NT < nel * D * NTB * 2) s_vt[tid + j * NT] = r_vt[j];
        }
    }
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    // the line operators are read with wave-uniform indices straight from the operator block
    // in global memory, through the constant address space (read-only for the whole launch:
    // scalar loads into SGPRs), so that the LDS carries only element data
    using CR = const __attribute__((address_space(4))) R;
    CR* cops = (CR*)a.ops;
    CR* lp = cops + op_lp(N);
    CR* cpv = cops + op_cp(N);
    const R* xi = &s_ops[op_xi(N)];
    // line units: unit u = wave + j NW covers direction k = u / WK (uniform in the wave) and
    // the lines (u % WK) 64 + lane of that direction: element el, + face point t
    auto for_units = [&](auto body) {
#pragma unroll
        for (int j = 0; j < UPW; ++j) {
            const int u = wave + j * S::NW;
            if (u >= S::NUNITS) break;
            const int k = u / S::WK;
            const int item = (u - k * S::WK) * 64 + lane;
            if (item >= nel * NFA) continue;
            const int el = item / NFA, t = item - el * NFA;
            if (k == 0) {
                body(std::integral_constant<int, 0>{}, j, el, t);
            } else if (k == 1) {
                body(std::integral_constant<int, 1>{}, j, el, t);
            } else if constexpr (D == 3) {
                body(std::integral_constant<int, 2>{}, j, el, t);
            }
        }
    };

    // ---- B1: corrected derivative along each line (Steps 1-3) ---------------------------
    R fu[UPW][V], fnb[UPW][V], fq[UPW][V];     // + face: own trace, neighbour trace, q_K
    for_units([&](auto KC, int j, int el, int t) {
        constexpr int K = decltype(KC)::value;
        constexpr int SK = st<N>(K);
        const int base = el * NU + face_base<D, N>(K, t);
        // the LDG jump (nb - own trace) is lifted, the own-trace part folded into
        // DT = D1 - cp (x) lp; on a + face without a neighbour (copy boundary: no jump) the
        // neighbour trace is taken as the own one, so that DT u + cp uf = D1 u and every line
        // applies the same, wave-uniform operator
        const bool hk = s_nbr[el * 2 * D + 2 * K + 1] >= 0;
        CR* Dm = cops + op_dt(N);
        const R jkk = AXIS ? s_geo[el * G + D + D * D + K * D + K] : R(1);
        R ul[V][N], nbv[V], uf[V], qf[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
#pragma unroll
            for (int q = 0; q < N; ++q) ul[v][q] = s_u[v][base + q * SK];
            uf[v] = R(0);
#pragma unroll
            for (int q = 0; q < N; ++q) uf[v] += lp[q] * ul[v][q];
            nbv[v] = hk ? s_nb[v][el * NPF + K * NFA + t] : uf[v];
            qf[v] = R(0);
        }
        // one operator row at a time, applied to both variables
#pragma unroll
        for (int q = 0; q < N; ++q) {
            R row[N];
#pragma unroll
            for (int b = 0; b < N; ++b) row[b] = Dm[q * N + b];
            const R c = cpv[q], l = lp[q];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R acc = R(0);
#pragma unroll
                for (int b = 0; b < N; ++b) acc += row[b] * ul[v][b];
                acc += c * nbv[v];
                const R qv = AXIS ? jkk * acc : acc;
                s_x[(v * D + K) * XST + base + q * SK] = qv;
                qf[v] += l * qv;
            }
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            fu[j][v] = uf[v];
            fnb[j][v] = nbv[v];
            fq[j][v] = qf[v];
        }
    });
    __syncthreads();

    // ---- B2: common normal flux on the + face points (Step 5) ----------------------------
    // velocity at reference position pos (node indices, N / N + 1 for the -1 / +1 end)
    auto vel_at = [&](int el, const int (&pos)[D], R (&vel)[D]) {
        const R* gg = &s_geo[el * G];
        if constexpr (AXIS) {
            if (trig) {
                velocity_tab<R, D, NTB>(a.ph, &s_vt[el * D * NTB * 2], pos, vel);
            } else {
                R x[D];
#pragma unroll
                for (int m = 0; m < D; ++m) {
                    const R xr = pos[m] == N ? R(0) : (pos[m] == N + 1 ? R(2) : xi[pos[m]] + R(1));
                    x[m] = gg[m] + gg[D + m * D + m] * xr;
                }
                velocity_lin<R, D>(a.ph, x, vel);
            }
        } else {
            R x[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                R acc = gg[i];
#pragma unroll
                for (int m = 0; m < D; ++m) {
                    const R xr = pos[m] == N ? R(0) : (pos[m] == N + 1 ? R(2) : xi[pos[m]] + R(1));
                    acc += gg[D + i * D + m] * xr;
                }
                x[i] = acc;
            }
            velocity<R, D>(a.ph, x, vel);
        }
    };
    // the common flux of face point t of face (K, SD) from its traces and gradient
    auto face_flux = [&](auto KC, auto SC, int el, int t, int32_t en, const R (&uL)[V],
                         const R (&uR)[V], const R (&qfa)[V][D]) {
        constexpr int K = decltype(KC)::value;
        constexpr int SD = decltype(SC)::value;
        const R* gg = &s_geo[el * G];
        R nrm[D], sc;
        if constexpr (AXIS) {
            const R jk = gg[D + D * D + K * D + K];
            sc = gg[D + 2 * D * D] * M::fabs_(jk);
#pragma unroll
            for (int i = 0; i < D; ++i) nrm[i] = R(0);
            nrm[K] = ((jk > R(0)) == (SD == 1)) ? R(1) : R(-1);
        } else {
            const R* fn = &s_fn[(el * D + K) * (D + 1)];
            sc = fn[D];
#pragma unroll
            for (int i = 0; i < D; ++i) nrm[i] = SD ? fn[i] : -fn[i];
        }
        R qn[V], g2 = R(0);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            R acc_n = R(0);
#pragma unroll
            for (int i = 0; i < D; ++i) {
                if constexpr (AXIS) {
                    if (i == K) acc_n = qfa[v][K] * nrm[K];
                } else {
                    acc_n += qfa[v][i] * nrm[i];
                }
                if (v == NV) g2 += qfa[v][i] * qfa[v][i];
            }
            qn[v] = acc_n;
        }
        int pos[D];
        {
            int tt = t;
#pragma unroll
            for (int m = 0; m < D; ++m) {
                if (m == K) {
                    pos[m] = N + SD;
                } else {
                    pos[m] = tt % N;
                    tt /= N;
                }
            }
        }
        R vel[D];
        vel_at(el, pos, vel);
        R v2 = R(0), vn = R(0);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            v2 += vel[i] * vel[i];
            if constexpr (AXIS) {
                if (i == K) vn = vel[K] * nrm[K];
            } else {
                vn += vel[i] * nrm[i];
            }
        }
        const R mm = max_sqrt(v2, a.ph.gamma);
        const R rn = M::rsqrt_(g2 + a.ph.delta_n * a.ph.delta_n);
        const R pL = uL[0], pR = uR[0], sL = uL[1], sR = uR[1];
        const R fvn = mm * (a.ph.eps * qn[0] - a.ph.gamma * pL * (R(1) - pL) * qn[NV] * rn);
        const R F0 = R(0.5) * (pL + pR) * vn - fvn + a.ph.tau * (pL - pR);
        const R F1 = R(0.5) * (sL + sR) * vn + a.ph.tau * (sL - sR);
        const uint32_t fo = (((uint32_t)(SD ? K : D + K)) * Eu + (uint32_t)(e0 + el)) * NFA + t;
        const R Fs0 = sc * F0, Fs1 = sc * F1;
        gst(a.Fp[0], fo, Fs0);
        gst(a.Fp[1], fo, Fs1);
        if constexpr (SD == 1) {
            // kept for the lifting of the + face in E1, in the slot of the neighbour trace
            // (read into registers in B1): the same thread writes and later reads it
            s_nb[0][el * NPF + K * NFA + t] = Fs0;
            s_nb[1][el * NPF + K * NFA + t] = Fs1;
        }
        (void)en;
    };
    // physical gradient at a face point from its interpolated reference (non-axis) or
    // physical (axis) components
    auto to_physical = [&](int el, const R (&qt)[D], R (&q)[D]) {
        if constexpr (AXIS) {
#pragma unroll
            for (int i = 0; i < D; ++i) q[i] = qt[i];
        } else {
            const R* Ji = &s_geo[el * G + D + D * D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                R acc = R(0);
#pragma unroll
                for (int k = 0; k < D; ++k) acc += Ji[k * D + i] * qt[k];
                q[i] = acc;
            }
        }
    };
    for_units([&](auto KC, int j, int el, int t) {
        constexpr int K = decltype(KC)::value;
        constexpr int SK = st<N>(K);
        const int base = el * NU + face_base<D, N>(K, t);
        const int32_t en = s_nbr[el * 2 * D + 2 * K + 1];
        R uL[V], uR[V], qfa[V][D];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            uL[v] = fu[j][v];
            uR[v] = (en >= 0) ? fnb[j][v] : fu[j][v];
            // the components other than K, interpolated to the face along the line (on
            // axis-aligned meshes only those of the interface normal's variable are needed)
            R qt[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                if (i == K) {
                    qt[i] = fq[j][v];
                } else if (!AXIS || v == NV) {
                    R acc = R(0);
#pragma unroll
                    for (int q = 0; q < N; ++q) acc += lp[q] * s_x[(v * D + i) * XST + base + q * SK];
                    qt[i] = acc;
                } else {
                    qt[i] = R(0);
                }
            }
            to_physical(el, qt, qfa[v]);
        }
        face_flux(KC, std::integral_constant<int, 1>{}, el, t, en, uL, uR, qfa);
    });
    // - faces on a boundary (face 2k without a neighbour): everything read from LDS along
    // the line, interpolated to the - end
    if (a.bnd_minus) {
        const R* lm = &s_ops[op_lm(N)];
        for_units([&](auto KC, int j, int el, int t) {
            (void)j;
            constexpr int K = decltype(KC)::value;
            constexpr int SK = st<N>(K);
            const int32_t en = s_nbr[el * 2 * D + 2 * K];
            if (en >= 0) return;
            const int base = el * NU + face_base<D, N>(K, t);
            R uL[V], qfa[V][D];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R acc = R(0);
#pragma unroll
                for (int q = 0; q < N; ++q) acc += lm[q] * s_u[v][base + q * SK];
                uL[v] = acc;
                R qt[D];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    R ai = R(0);
#pragma unroll
                    for (int q = 0; q < N; ++q) ai += lm[q] * s_x[(v * D + i) * XST + base + q * SK];
                    qt[i] = ai;
                }
                to_physical(el, qt, qfa[v]);
            }
            face_flux(KC, std::integral_constant<int, 0>{}, el, t, en, uL, uL, qfa);
        });
    }

    // the point fluxes below overwrite the gradient the face phase reads along lines
    __syncthreads();

    // solution-point phases: one pass when the block has a thread per point, else a loop
    // over the block's points
    auto for_points = [&](auto body) {
        if constexpr (NT >= EPB * NU) {
            if (tid < nel * NU) body(tid);
        } else {
            for (int tp = tid; tp < nel * NU; tp += NT) body(tp);
        }
    };

    // ---- B2: fluxes at the solution points (Step 4) --------------------------------------
    for_points([&](const int tp) {
        const int le = tp / NU, ip = tp - le * NU;
        const R* gg = &s_geo[le * G];
        const R det = gg[D + 2 * D * D];
        const R* Ji = gg + D + D * D;            // Jinv[k][i] = Ji[k*D + i]
        int mi[D];
        {
            int r = ip;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                mi[k] = r % N;
                r /= N;
            }
        }
        R q[V][D];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            R qt[D];
#pragma unroll
            for (int i = 0; i < D; ++i) qt[i] = s_x[(v * D + i) * XST + tp];
            to_physical(le, qt, q[v]);
        }
        R vel[D];
        vel_at(le, mi, vel);
        R v2 = R(0), g2 = R(0);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            v2 += vel[i] * vel[i];
            g2 += q[NV][i] * q[NV][i];
        }
        const R mm = max_sqrt(v2, a.ph.gamma);
        const R rn = M::rsqrt_(g2 + a.ph.delta_n * a.ph.delta_n);
        const R phi = s_u[0][tp], psi = s_u[1][tp];
        const R sharp = a.ph.gamma * phi * (R(1) - phi) * rn;
        R f0[D], f1[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const R fvis = mm * (a.ph.eps * q[0][i] - sharp * q[NV][i]);
            f0[i] = phi * vel[i] - fvis;
            f1[i] = psi * vel[i];
        }
#pragma unroll
        for (int k = 0; k < D; ++k) {
            R a0, a1;
            if constexpr (AXIS) {
                a0 = Ji[k * D + k] * f0[k];
                a1 = Ji[k * D + k] * f1[k];
            } else {
                a0 = R(0);
                a1 = R(0);
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    a0 += Ji[k * D + i] * f0[i];
                    a1 += Ji[k * D + i] * f1[i];
                }
            }
            s_x[(0 * D + k) * XST + tp] = det * a0;
            s_x[(1 * D + k) * XST + tp] = det * a1;
        }
    });
    __syncthreads();

    // ---- E1: DH_K f~_K along each line (volume part of Step 6), in place, plus the
    // lifting cp F~ of the line's + face common flux (the face part of Step 6 on the faces
    // this element owns; the update adds the - faces') ----------------------------------
    CR* DH = cops + op_dh(N);
    for_units([&](auto KC, int j, int el, int t) {
        (void)j;
        constexpr int K = decltype(KC)::value;
        constexpr int SK = st<N>(K);
        const int base = el * NU + face_base<D, N>(K, t);
        R fl[V][N], fp[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
#pragma unroll
            for (int b = 0; b < N; ++b) fl[v][b] = s_x[(v * D + K) * XST + base + b * SK];
            fp[v] = s_nb[v][el * NPF + K * NFA + t];
        }
#pragma unroll
        for (int q = 0; q < N; ++q) {
            R row[N];
#pragma unroll
            for (int b = 0; b < N; ++b) row[b] = DH[q * N + b];
            const R c = cpv[q];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                R acc = R(0);
#pragma unroll
                for (int b = 0; b < N; ++b) acc += row[b] * fl[v][b];
                s_x[(v * D + K) * XST + base + q * SK] = acc + c * fp[v];
            }
        }
    });
    __syncthreads();

    // ---- E2: P = sum over the directions ------------------------------------------------
    for_points([&](const int tp) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            R acc = R(0);
#pragma unroll
            for (int k = 0; k < D; ++k) acc += s_x[(v * D + k) * XST + tp];
            gst_s<STREAM>(a.P[v] + e0 * NU, (uint32_t)tp, acc);
        }
    });
}

// ------------------------------------------------------------------------------------
// - face traces of the block's elements pushed into the owners' + face slots. Face unit
// j of a wave covers direction k = u / WK, points (u % WK) * 64 + lane of that direction
// (u = wave + j NW), so the direction is uniform in the wave.
// ------------------------------------------------------------------------------------
template <int D, int P, int U, typename S = Shape<D, P>>
__device__ __forceinline__ void load_owners(int32_t (&r_own)[U], const int32_t* nbr, int64_t e0,
                                            int nel, int wave, int lane) {
#pragma unroll
    for (int j = 0; j < S::UPW; ++j) {
        const int u = wave + j * S::NW;
        r_own[j] = -1;
        if (u < S::NUNITS) {
            const int k = u / S::WK;
            const int item = (u - k * S::WK) * 64 + lane;
            if (item < nel * S::NFA) r_own[j] = gld(nbr + e0 * 2 * D, (item / S::NFA) * 2 * D + 2 * k);
        }
    }
}

template <typename R, int D, int P, int V, int U, typename S = Shape<D, P>>
__device__ __forceinline__ void push_traces(R* const* Tp, const R* lm, const R* su0,
                                            const R* su1, const int32_t (&r_own)[U], int nel,
                                            int wave, int lane, uint32_t E) {
    constexpr int N = S::N, NU = S::NU, NFA = S::NFA;
    auto push = [&](auto KC, int el, int t, int32_t own) {
        constexpr int K = decltype(KC)::value;
        constexpr int SK = st<N>(K);
        const int base = el * NU + face_base<D, N>(K, t);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const R* su = v ? su1 : su0;
            R acc = R(0);
#pragma unroll
            for (int q = 0; q < N; ++q) acc += lm[q] * su[base + q * SK];
            gst(Tp[v], ((uint32_t)K * E + (uint32_t)own) * NFA + t, acc);
        }
    };
#pragma unroll
    for (int j = 0; j < S::UPW; ++j) {
        const int u = wave + j * S::NW;
        if (u >= S::NUNITS) break;
        const int k = u / S::WK;
        const int item = (u - k * S::WK) * 64 + lane;
        if (item >= nel * NFA || r_own[j] < 0) continue;
        const int el = item / NFA, t = item - el * NFA;
        if (k == 0) {
            push(std::integral_constant<int, 0>{}, el, t, r_own[j]);
        } else if (k == 1) {
            push(std::integral_constant<int, 1>{}, el, t, r_own[j]);
        } else if constexpr (D == 3) {
            push(std::integral_constant<int, 2>{}, el, t, r_own[j]);
        }
    }
}

// ------------------------------------------------------------------------------------
// update: Step 6 face part and the RK4 stage combine.
//   R = -(P + sum_faces c_face F~) / |J|; then either the residual is written (UP_RESID)
//   or the classic RK4 registers are advanced and the - face traces of the next stage
//   input are written (UP_RK).
// ------------------------------------------------------------------------------------
// STREAM: the state planes are larger than the caches (more than XCD_MAP_MAX_PLANE_BYTES
// each); the registers read and written once per stage (P, u_n, the accumulator, the next
// stage input) then go with the non-temporal hint.
// PF: P already holds the lifting of the element's + face fluxes (the line kernel adds it,
// from the fluxes it has just computed); only the - face fluxes are read here.
template <typename R, int D, int P, int V, int KIND, bool STREAM, bool PF>
__global__ __launch_bounds__((Shape<D, P, update_tpb(D, P, sizeof(R))>::NT))
void k_update(UPArgs<R> a) {
    using S = Shape<D, P, update_tpb(D, P, sizeof(R))>;
    constexpr int N = S::N, NU = S::NU, NFA = S::NFA, EPB = S::EPB, NT = S::NT, G = S::GEO;
    constexpr int NFS = PF ? D : 2 * D;      // faces whose fluxes are read, per element
    constexpr int NFE = NFS * NFA;
    __shared__ R s_c[3 * N];                 // cm, cp, lm
    __shared__ R s_F[V][EPB * NFE];
    __shared__ R s_u[V][KIND == UP_RK ? EPB * NU : 1];

    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)block_chunk<R>(a.E * NU) * EPB;
    const int nel = (int)((a.E - e0) < EPB ? (a.E - e0) : EPB);
    const bool pt = tid < nel * NU;
    const int le = tid / NU;
    const int ip = tid - le * NU;
    // every global load is issued before the first wait; all are indexed by this block's
    // own elements (the owners pushed the - face fluxes here). The adjacency is only needed
    // for the addresses of the trace pushes at the end.
    constexpr int I_F = (EPB * NFE + NT - 1) / NT;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    int32_t r_own[S::UPW];
    if constexpr (KIND == UP_RK) load_owners<D, P, S::UPW, S>(r_own, a.nbr, e0, nel, wave, lane);
    R rP[V], rU[V], rA[V];
    const uint32_t so = e0 * NU;     // first state value of the block (per plane)
    // lanes past the block's points load its last point (values unused)
    const int tp = pt ? tid : nel * NU - 1;
    const R det = gld(a.geo + e0 * G, (tp / NU) * G + D + 2 * D * D);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        rP[v] = gld_s<STREAM>(a.P[v] + so, (uint32_t)tp);
        if constexpr (KIND == UP_RK) {
            rU[v] = gld_s<STREAM>(a.un[v] + so, (uint32_t)tp);
            rA[v] = a.first ? R(0) : gld_s<STREAM>(a.acc[v] + so, (uint32_t)tp);
        }
    }
    R r_c[3];
    r_c[0] = gld_in(a.ops + op_cm(N), tid, N);
    r_c[1] = gld_in(a.ops + op_cp(N), tid, N);
    r_c[2] = gld_in(a.ops + op_lm(N), tid, N);
    // lanes run over [face f][el NFA + t], f = 2k + s (f = k, the - faces only, with PF):
    // the + face fluxes of the block are contiguous in plane k; the - face flux is minus the
    // owner's + face flux in plane k (the owners e - stride_k of consecutive elements are
    // consecutive), or on a boundary the element's own, in plane D + k
    constexpr int KSEG = S::KSEG;
    const uint32_t Eu = (uint32_t)a.E;
    R r_F[I_F][V];
    int f_pos[I_F];
    bool f_neg[I_F];
#pragma unroll
    for (int j = 0; j < I_F; ++j) {
        const int it = tid + j * NT;
        int f = it / KSEG;
        int r = it - f * KSEG;
        const bool ok = f < NFS && r < nel * NFA;
        f = f < NFS ? f : NFS - 1;
        r = r < nel * NFA ? r : nel * NFA - 1;
        const int el = r / NFA, t = r - el * NFA;
        const int k = PF ? f : f >> 1, sd = PF ? 0 : f & 1;
        f_pos[j] = ok ? el * NFE + f * NFA + t : -1;
        uint32_t gi;
        bool neg = false;
        if (sd) {
            gi = ((uint32_t)k * Eu + (uint32_t)e0) * NFA + (uint32_t)r;
        } else {
            const int32_t en = gld(a.nbr, (uint32_t)((e0 + el) * 2 * D + 2 * k));
            neg = en >= 0;
            gi = neg ? ((uint32_t)k * Eu + (uint32_t)en) * NFA + t
                     : ((uint32_t)(D + k) * Eu + (uint32_t)(e0 + el)) * NFA + t;
        }
        f_neg[j] = neg;
#pragma unroll
        for (int v = 0; v < V; ++v) r_F[j][v] = gld(a.Fp[v], gi);
    }
    if (tid < N) {
        s_c[tid] = r_c[0];
        s_c[N + tid] = r_c[1];
        s_c[2 * N + tid] = r_c[2];
    }
#pragma unroll
    for (int j = 0; j < I_F; ++j)
        if (f_pos[j] >= 0)
#pragma unroll
            for (int v = 0; v < V; ++v) s_F[v][f_pos[j]] = f_neg[j] ? -r_F[j][v] : r_F[j][v];
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
        const R rdet = R(1) / det;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            R acc = rP[v];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int tk = tang_index<D, N>(k, mi);
                if constexpr (PF)
                    acc += s_c[mi[k]] * s_F[v][le * NFE + k * NFA + tk];
                else
                    acc += s_c[N + mi[k]] * s_F[v][le * NFE + (2 * k + 1) * NFA + tk]
                         + s_c[mi[k]] * s_F[v][le * NFE + (2 * k) * NFA + tk];
            }
            const R res = -acc * rdet;
            if constexpr (KIND == UP_RESID) {
                gst_s<STREAM>(a.res[v] + so, (uint32_t)tid, res);
            } else {
                // explicit fused multiply-adds: one rounding per register update, whatever
                // the surrounding code lets the compiler contract
                using M = Math<R>;
                R nx;
                if (!a.last) {
                    gst_s<STREAM>(a.acc[v] + so, (uint32_t)tid, M::fma_(a.bcoef, res, rA[v]));
                    nx = M::fma_(a.ccoef, res, rU[v]);
                    gst_s<STREAM>(a.us[v] + so, (uint32_t)tid, nx);
                } else {
                    nx = M::fma_(a.ccoef, M::fma_(a.bcoef, res, rA[v]), rU[v]);
                    gst_s<STREAM>(a.un[v] + so, (uint32_t)tid, nx);
                    if (a.uo[0]) gst_s<STREAM>(a.uo[v] + so, (uint32_t)tid, nx);
                }
                s_u[v][tid] = nx;
                const R lim = (v == 0 && V == 2) ? R(10) : R(1e30);
                if (!(Math<R>::fabs_(nx) <= lim)) *a.flag = 1;
            }
        }
    }
    if constexpr (KIND == UP_RK) {
        __syncthreads();
        // - face traces of the next stage input, pushed into the owners' + face slots
        push_traces<R, D, P, V, S::UPW, S>(a.Tp, &s_c[2 * N], s_u[0], s_u[V - 1], r_own, nel, wave,
                                           lane, (uint32_t)a.E);
    }
}

// - face traces of a given state pushed into the owners' + face slots (after set_state /
// reset)
template <typename R, int D, int P, int V>
__global__ __launch_bounds__((Shape<D, P>::NT)) void k_trace(TRArgs<R> a) {
    using S = Shape<D, P>;
    constexpr int N = S::N, NU = S::NU, EPB = S::EPB, NT = S::NT;
    constexpr int I_U = (EPB * NU + NT - 1) / NT;
    __shared__ R s_lm[N];
    __shared__ R s_u[V][EPB * NU];
    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)block_chunk<R>(a.E * NU) * EPB;
    const int nel = (int)((a.E - e0) < EPB ? (a.E - e0) : EPB);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    int32_t r_own[S::UPW];
    load_owners<D, P, S::UPW>(r_own, a.nbr, e0, nel, wave, lane);
    R r_u[V][I_U];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
        for (int j = 0; j < I_U; ++j) {
            const int i = tid + j * NT;
            r_u[v][j] = (i < nel * NU) ? gld(a.u[v] + e0 * NU, i) : R(0);
        }
    R r_l = (tid < N) ? gld(a.ops + op_lm(N), tid) : R(0);
    if (tid < N) s_lm[tid] = r_l;
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
        for (int j = 0; j < I_U; ++j)
            if (tid + j * NT < nel * NU) s_u[v][tid + j * NT] = r_u[v][j];
    __syncthreads();
    push_traces<R, D, P, V, S::UPW>(a.Tp, s_lm, s_u[0], s_u[V - 1], r_own, nel, wave, lane,
                                    (uint32_t)a.E);
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
        if (a.kind == 2) {
            const double df = f - (double)a.ref[idx];
            acc += df * df;
            continue;
        }
        if (a.kind == 1) f = ::fabs(f - (double)a.ref[idx]);
        acc += a.det64[e] * W * f;
    }
    const double b = block_sum(acc);
    if (threadIdx.x == 0) a.partial[blockIdx.x] = b;
}

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------
template <typename R, int D, int P>
struct Impl {
    using S = Shape<D, P>;
    static unsigned grid(int64_t E) { return (unsigned)((E + S::EPB - 1) / S::EPB); }
    // the line kernel runs the physical mode, outside the BF16 form, in 3D, and in 2D in
    // FP32 (128^2 p4: FP32 grad_flux 6.9 -> 6.2 us) and in FP64 from p = 4 (128^2 p4 with
    // the operators in SGPRs and the + face lifting: 0.0763 -> 0.0720 ms/step; at 64^2 p3
    // the point kernel stays ahead, 0.0307 against 0.0319)
    static constexpr bool LINES_DIM = D == 3 || sizeof(R) == 4 || P >= 4;
    static constexpr bool lines(int mode, bool mf) { return mode == GF_PHYS && !mf && LINES_DIM; }

    template <int MODE, bool AXIS, bool MF, bool NPHI>
    static void gf_launch(const GFArgs<R>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
        if constexpr (lines(MODE, MF)) {
            constexpr int NTL = lines_nt<R, D, P>();
            if (a.E * S::NU * (int64_t)sizeof(R) > XCD_MAP_MAX_PLANE_BYTES)
                hipExtLaunchKernelGGL((k_grad_flux_lines<R, D, P, AXIS, NPHI, true>), dim3(grid(a.E)),
                                      dim3(NTL), 0, st, e0, e1, 0, a);
            else
                hipExtLaunchKernelGGL((k_grad_flux_lines<R, D, P, AXIS, NPHI, false>), dim3(grid(a.E)),
                                      dim3(NTL), 0, st, e0, e1, 0, a);
        } else {
            hipExtLaunchKernelGGL((k_grad_flux<R, D, P, MODE, AXIS, MF, NPHI>), dim3(grid(a.E)),
                                  dim3(S::NT), 0, st, e0, e1, 0, a);
        }
    }
    template <int MODE, bool MF>
    static void gf_mode(const GFArgs<R>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
        if constexpr (MODE == GF_PHYS) {
            if (a.axis) {
                if (a.nphi) gf_launch<MODE, true, MF, true>(a, st, e0, e1);
                else gf_launch<MODE, true, MF, false>(a, st, e0, e1);
            } else {
                if (a.nphi) gf_launch<MODE, false, MF, true>(a, st, e0, e1);
                else gf_launch<MODE, false, MF, false>(a, st, e0, e1);
            }
        } else if constexpr (MODE == GF_PRECOND) {
            if (a.axis) gf_launch<MODE, true, MF, false>(a, st, e0, e1);
            else gf_launch<MODE, false, MF, false>(a, st, e0, e1);
        } else {
            gf_launch<MODE, false, MF && MODE != GF_SENSOR, false>(a, st, e0, e1);
        }
    }
    template <bool MF>
    static void gf_dispatch(int mode, const GFArgs<R>& a, hipStream_t st, hipEvent_t e0,
                            hipEvent_t e1) {
        switch (mode) {
            case GF_PHYS: gf_mode<GF_PHYS, MF>(a, st, e0, e1); break;
            case GF_PRECOND: gf_mode<GF_PRECOND, MF>(a, st, e0, e1); break;
            case GF_SIGN: gf_mode<GF_SIGN, MF>(a, st, e0, e1); break;
            default: gf_mode<GF_SENSOR, MF>(a, st, e0, e1); break;
        }
    }
    static void grad_flux(int mode, int nvar, const GFArgs<R>& a, hipStream_t st, hipEvent_t e0,
                          hipEvent_t e1) {
        (void)nvar;
        if constexpr (std::is_same<R, float>::value) {
            if (a.mf) {
                gf_dispatch<true>(mode, a, st, e0, e1);
                return;
            }
        }
        gf_dispatch<false>(mode, a, st, e0, e1);
    }
    static void update(int kind, int nvar, const UPArgs<R>& a, hipStream_t st, hipEvent_t e0,
                       hipEvent_t e1) {
        using U = Shape<D, P, update_tpb(D, P, sizeof(R))>;
        const dim3 g((unsigned)((a.E + U::EPB - 1) / U::EPB)), b(U::NT);
        const bool stream = a.E * S::NU * (int64_t)sizeof(R) > XCD_MAP_MAX_PLANE_BYTES;
        // two variables: the physical mode, whose grad_flux may be the line kernel (which
        // has lifted the + face fluxes into P already); one variable: preconditioning
        const bool pf = nvar == 2 && lines(GF_PHYS, a.mf != 0);
        auto go = [&](auto STC, auto PFC) {
            constexpr bool ST = decltype(STC)::value, PF = decltype(PFC)::value;
            if (nvar == 2) {
                if (kind == UP_RK) hipExtLaunchKernelGGL((k_update<R, D, P, 2, UP_RK, ST, PF>), g, b, 0, st, e0, e1, 0, a);
                else hipExtLaunchKernelGGL((k_update<R, D, P, 2, UP_RESID, ST, PF>), g, b, 0, st, e0, e1, 0, a);
            } else if constexpr (!PF) {
                if (kind == UP_RK) hipExtLaunchKernelGGL((k_update<R, D, P, 1, UP_RK, ST, false>), g, b, 0, st, e0, e1, 0, a);
                else hipExtLaunchKernelGGL((k_update<R, D, P, 1, UP_RESID, ST, false>), g, b, 0, st, e0, e1, 0, a);
            }
        };
        auto go_pf = [&](auto STC) {
            if constexpr (LINES_DIM) {
                if (pf) {
                    go(STC, std::true_type{});
                    return;
                }
            }
            go(STC, std::false_type{});
        };
        if (stream) go_pf(std::true_type{});
        else go_pf(std::false_type{});
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

// Launch table of one (d, p) for the orders built for dimension D (defined here, explicitly
// instantiated once per dimension and precision).
template <typename R, int D>
bool get_launchers_dim(int p, Launchers<R>* L) {
    switch (p) {
        case 1: return fill<R, D, 1>(L);
        case 2: return fill<R, D, 2>(L);
        case 3: return fill<R, D, 3>(L);
        case 4: return fill<R, D, 4>(L);
        case 5: return fill<R, D, 5>(L);
        case 6:
            if constexpr (D == 2) return fill<R, D, 6>(L);
            return false;
        default: return false;
    }
}

}  // namespace pcpf
