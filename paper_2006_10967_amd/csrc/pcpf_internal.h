// Internal declarations shared by the HIP kernels and the C-ABI implementation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "pcpf.h"

namespace pcpf {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// Block shape of the forward kernels for a (d, p) element: one thread per solution point,
// EPB = floor(TPB / N_u) whole elements per block (at least one), NT = EPB N_u rounded up
// to whole 64-wide waves. The face phases split the block's face points by reference
// direction into units of one wave (KSEG = EPB N_fa points per direction, WK waves each),
// so that the direction, and with it every stride of the face code, is uniform in a wave.
template <int D, int P, int TPB = 256, int NTO = 0>
struct Shape {
    static constexpr int N = P + 1;
    static constexpr int NU = ipow(N, D);
    static constexpr int NFA = ipow(N, D - 1);
    static constexpr int NF = 2 * D * NFA;
    static constexpr int EPB = (TPB / NU) >= 1 ? TPB / NU : 1;
    static constexpr int NT = NTO ? NTO : (EPB * NU + 63) / 64 * 64;
    static constexpr int NW = NT / 64;
    static constexpr int KSEG = EPB * NFA;
    static constexpr int WK = (KSEG + 63) / 64;
    static constexpr int NUNITS = D * WK;
    static constexpr int UPW = (NUNITS + NW - 1) / NW;   // face units per wave
    static constexpr int GEO = D + 2 * D * D + 1;   // x0[D], J[D][D], Jinv[D][D], detJ
};

// Threads per block of the line kernel. 3D in FP32: one wave per unit of line work (D WK
// waves), the solution-point phases looping over the block's points where those exceed the
// threads, so that no wave of a block idles through the line phases (96^3 p4 grad_flux
// 1135 -> 1103 us, 64^3 p3 146 -> 141 us). FP64 keeps a thread per point: with three waves
// per block it lost (2054 -> 2072 us, 262 -> 284 us).
template <typename R, int D, int P>
constexpr int lines_nt() {
    using S = Shape<D, P>;
    return (D == 3 && sizeof(R) == 4 && 64 * S::NUNITS < S::NT) ? 64 * S::NUNITS : S::NT;
}

// Threads per block of the update kernel: for the 3D elements of 125 or more points in FP64,
// 1024 (eight elements per block, so that the runs a block reads and writes in each face
// plane span eight elements: 96^3 p4 2274 us at 256, 2206 at 512, 2056 at 1024, before
// the per-XCD runs of chunks; with them 512 and 1024 are within 0.5 %); 256 otherwise
// (FP32 96^3 p4 with the per-XCD runs: 992 us at 256, 1031 at 512, 1075 at 1024; no gain
// from larger blocks at 64 points).
constexpr int update_tpb(int d, int p, int word) {
    return (d == 3 && p >= 4 && word == 8) ? 1024 : 256;
}

// Lane utilisation (per mille) of nt-thread blocks holding whole elements of nu points.
constexpr int lane_util(int nu, int nt) { return nt >= nu ? (nt / nu) * nu * 1000 / nt : 0; }
// Smallest block (64, 128 or 256 threads) that keeps >= 90% of the lanes busy, else the
// best of the three.
constexpr int pick_nt(int nu) {
    return lane_util(nu, 64) >= 900    ? 64
           : lane_util(nu, 128) >= 900 ? 128
           : lane_util(nu, 256) >= 900 ? 256
           : (lane_util(nu, 128) >= lane_util(nu, 256) ? 128 : 256);
}

// Block shape of the adjoint kernels: one thread per solution point in the smallest block
// that keeps >= 90% of the lanes busy.
template <int D, int P>
struct AShape {
    static constexpr int N = P + 1;
    static constexpr int NU = ipow(N, D);
    static constexpr int NFA = ipow(N, D - 1);
    static constexpr int NF = 2 * D * NFA;
    static constexpr int NT = pick_nt(NU);
    static constexpr int EPB = NT / NU;
    static constexpr int GEO = D + 2 * D * D + 1;
};

// Operator block (compute type), n = p + 1:
//   D1[n*n]  nodal derivative;
//   DH[n*n]  D1 - cp (x) lp + cm (x) lm: derivative minus the lifted discontinuous normal
//            flux of both ends (volume part of the corrected divergence);
//   DT[n*n]  D1 - cp (x) lp: derivative minus the lifted own trace of the + end (with the
//            neighbour's trace lifted separately this is the corrected gradient of a line
//            whose + face has a neighbour);
//   VINV[n*n], lm[n], lp[n], cm[n], cp[n], xi[n], w[n]
constexpr int ops_size(int n) { return 4 * n * n + 6 * n; }
constexpr int OP_D1 = 0;
constexpr int op_dh(int n) { return n * n; }
constexpr int op_vinv(int n) { return 2 * n * n; }
constexpr int op_dt(int n) { return 3 * n * n; }
constexpr int op_lm(int n) { return 4 * n * n; }
constexpr int op_lp(int n) { return 4 * n * n + n; }
constexpr int op_cm(int n) { return 4 * n * n + 2 * n; }
constexpr int op_cp(int n) { return 4 * n * n + 3 * n; }
constexpr int op_xi(int n) { return 4 * n * n + 4 * n; }
constexpr int op_w(int n) { return 4 * n * n + 5 * n; }

// kernel-side physics parameters (compute type)
template <typename R>
struct Phys {
    R gamma, eps, tau, delta_n, delta_g, nu_max, s0, kappa;
    R ampg;        // A * g(t) at the stage time
    R u0[3];
    int vel_kind;
};

// grad_flux kernel modes
enum { GF_PHYS = 0, GF_PRECOND = 1, GF_SIGN = 2, GF_SENSOR = 3 };

template <typename R>
struct GFArgs {
    const R* u[2];       // stage input per variable ([E][NU])
    R* P[2];             // partial divergence per variable
    R* Fp[2];            // common fluxes per variable, [2D][E][NFA]: plane k < D the flux of
                         // the + face k (its owner's), plane D + k the flux of the - face k
                         // where it lies on a boundary (written only there)
    const R* Tp[2];      // neighbour traces on the own + faces (pushed), [D][E][NFA]
    const R* geo;        // [E][GEO]
    const int32_t* nbr;  // [E][2D]
    const R* ops;
    const R* sgn;        // smeared sign (precond)
    const R* vtab;       // sin^2(pi x_k), sin(2 pi x_k) at the n nodes and both ends of
                         // every element axis, [E][D][n + 2][2] (axis-aligned
                         // trigonometric fields)
    R* out;              // sign (GF_SIGN) or nu (GF_SENSOR)
    int64_t E;
    Phys<R> ph;
    int axis;            // every element axis-aligned (diagonal J): diagonal-Jacobian
                         // arithmetic and velocity from per-element 1D sin/cos tables
    int mf;              // line operators on the matrix cores, bf16 operands (float only)
    int nphi;            // interface normal from phi (the unpreconditioned form)
    int sgn_current;     // GF_PRECOND: sgn holds psi0 and the sign is tanh(psi0 / |grad psi|)
                         // of the current stage
    int bnd_minus;       // some - face of the mesh lies on a boundary (its flux is computed
                         // by the element itself)
};

// update kernel kinds
enum { UP_RK = 0, UP_RESID = 1 };

template <typename R>
struct UPArgs {
    const R* P[2];
    const R* Fp[2];      // common fluxes [2D][E][NFA] (as GFArgs::Fp); the flux of an interior
                         // - face is minus the owner's + face flux
    R* un[2];            // u_n (read; written on the last stage)
    R* uo[2];            // null, or a second destination of u_{n+1} on the last stage
    R* acc[2];           // RK accumulator
    R* us[2];            // next stage input (written on stages 0-2)
    R* res[2];           // residual output (UP_RESID)
    R* Tp[2];            // - face traces of the next stage input, pushed to the owners'
                         // + face slots, [D][E][NFA]
    const R* geo;
    const int32_t* nbr;
    const R* ops;
    int* flag;           // set to 1 on a non-finite value or |phi| > 10
    int64_t E;
    R bcoef;             // weight of R in the accumulator
    R ccoef;             // step of the next stage input (a_{s+1} dt), or dt on the last stage
    int first, last;
    int mf;              // as GFArgs::mf: selects which grad_flux kernel produced P (the line
                         // kernel also lifts the + face fluxes into P)
};

template <typename R>
struct TRArgs {
    const R* u[2];
    R* Tp[2];
    const int32_t* nbr;
    const R* ops;
    int64_t E;
};

template <typename R>
struct RDArgs {
    const R* field;
    const R* ref;        // may be null
    const double* det64; // |J| per element in float64
    const double* w64;   // 1D quadrature weights in float64
    double* partial;
    int64_t E;
    int kind;            // 0 mass, 1 L1, 2 unweighted sum of (field - ref)^2
};

// Launch table of one (precision, d, p) instantiation.
template <typename R>
struct Launchers {
    int epb, nt, ngeo;
    // ev0/ev1 (may be null): events the dispatch itself records at kernel start and end
    void (*grad_flux)(int mode, int nvar, const GFArgs<R>&, hipStream_t, hipEvent_t ev0,
                      hipEvent_t ev1);
    void (*update)(int kind, int nvar, const UPArgs<R>&, hipStream_t, hipEvent_t ev0,
                   hipEvent_t ev1);
    void (*trace)(int nvar, const TRArgs<R>&, hipStream_t);
    void (*reduce)(const RDArgs<R>&, int nblocks, hipStream_t);
};

template <typename R>
bool get_launchers(int d, int p, Launchers<R>* out);

// elementwise helpers (not order dependent)
template <typename R>
void launch_reset(const R* phi, R* psi, int64_t n, int mode, double eps_w, double delta_phi,
                  hipStream_t s);
void launch_reduce_final(const double* partial, int nblocks, double* out, hipStream_t s);

constexpr int REDUCE_BLOCKS = 1024;
constexpr int REDUCE_THREADS = 256;

}  // namespace pcpf
