// Adjoint kernels: argument blocks and launch table.
#pragma once

#include "pcpf_internal.h"

namespace pcpf {

enum { AD_PHYS = 0, AD_PRECOND = 1, AD_SIGN = 2 };

template <typename R>
struct AJPush {
    const R* rbar[2];    // R^ of the stage (per variable, [E][NU])
    R* gp[2];            // out: flux adjoints pushed into the owners' + face slots
    const R* u[2];       // stage input Y
    R* Tp[2];            // out: forward - face traces of Y pushed into the owners' + face slots
    const R* geo;
    const int32_t* nbr;
    const R* ops;
    int64_t E;
    // start of a reverse step (seed_yb set): R^ is not read but formed as seed_alpha * yb
    // and written to seed_rb, and seed_ya receives a copy of yb
    const R* seed_yb[2];
    R* seed_ya[2];
    R* seed_rb[2];
    R seed_alpha;
};

template <typename R>
struct AJMain {
    const R* u[2];       // stage input Y
    const R* Tp[2];      // forward neighbour traces of Y in the + face slots
    const R* rbar[2];    // R^ (residual modes)
    const R* gp[2];      // pushed flux adjoints of the own + faces
    R* ub[2];            // out: own part of Y^
    R* tb[2];            // out: trace adjoints pushed into the neighbours' - face slots
    R* sb;               // precond: sign adjoint accumulator (+=); sign mode: the sign adjoint
    const R* sgn;        // smeared sign (precond and sign modes)
    const R* geo;
    const int32_t* nbr;
    const R* ops;
    double* apart;       // per-block dL/dA partial sums (+=, physical mode)
    int64_t E;
    Phys<R> ph;
    R amp;               // velocity amplitude A
    R gt;                // time factor g(t): v = A g(t) v0(x)
};

template <typename R>
struct AJFinish {
    const R* ub[2];
    const R* tb[2];
    R* ya[2];            // += Y^ (may be null)
    R* rnext[2];         // = c_prev * yb + c_cur * Y^ (may be null)
    const R* yb[2];
    const int32_t* nbr;
    const R* ops;
    int64_t E;
    R c_prev, c_cur;
    // optional: the push of the next (earlier) stage, whose R^ is rnext, run after the
    // combine (ynext set; rnext must be set then)
    const R* ynext[2];   // that stage's input Y
    R* gp[2];
    R* Tp[2];
    const R* geo;
};

template <typename R>
struct AdjLaunchers {
    int epb;             // elements per block of the adjoint kernels (partial sums per block)
    void (*push)(int nvar, const AJPush<R>&, hipStream_t);
    void (*main)(int mode, const AJMain<R>&, hipStream_t);
    void (*finish)(int nvar, const AJFinish<R>&, hipStream_t);
};

template <typename R>
bool get_adj_launchers(int d, int p, AdjLaunchers<R>* out);
template <typename R>
void launch_reset_adj(R* phib, const R* psi0b, const R* phi, int64_t n, int mode, double eps_w,
                      double dphi, hipStream_t s);
template <typename R>
void launch_loss_seed(R* out, const R* phi, const R* target, const R* geo, const R* w, int64_t E,
                      int nu, int n, int d, hipStream_t s);

}  // namespace pcpf
