/* The C ABI of include/pcpf.h used from plain C99 (host calls only: no GPU needed).
 * Checks the 1D operators of the Gauss-Legendre element against facts of the element
 * (weights sum to the reference length, the derivative of a constant is 0 and of xi is 1,
 * the end interpolations reproduce xi at +-1, the DG correction divergences equal
 * l(+-1)/w), the solution coordinates of an affine box element, the workspace size query
 * and the error path. Prints one line per check and returns the number of failures. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "pcpf.h"

static int fails = 0;

static void check(int ok, const char* what) {
    printf("%s %s\n", ok ? "ok  " : "FAIL", what);
    if (!ok) ++fails;
}

int main(void) {
    enum { P = 3, N = P + 1 };
    double nodes[N], w[N], D[N * N], lm[N], lp[N], cm[N], cp[N], vinv[N * N];
    check(pcpf_abi_version() == PCPF_ABI_VERSION, "abi version");
    check(pcpf_line_operators(P, nodes, w, D, lm, lp, cm, cp, vinv) == PCPF_OK, "line operators");
    double sw = 0.0, lpx = 0.0, lmx = 0.0, worst_d0 = 0.0, worst_d1 = 0.0, worst_c = 0.0;
    for (int a = 0; a < N; ++a) {
        sw += w[a];
        lpx += lp[a] * nodes[a];
        lmx += lm[a] * nodes[a];
        double r0 = 0.0, r1 = 0.0;
        for (int b = 0; b < N; ++b) {
            r0 += D[a * N + b];
            r1 += D[a * N + b] * nodes[b];
        }
        worst_d0 = fmax(worst_d0, fabs(r0));
        worst_d1 = fmax(worst_d1, fabs(r1 - 1.0));
        worst_c = fmax(worst_c, fabs(cp[a] - lp[a] / w[a]) + fabs(cm[a] - lm[a] / w[a]));
    }
    check(fabs(sw - 2.0) < 1e-14, "weights sum to 2");
    check(worst_d0 < 1e-13 && worst_d1 < 1e-13, "derivative exact on 1 and xi");
    check(fabs(lpx - 1.0) < 1e-14 && fabs(lmx + 1.0) < 1e-14, "end interpolation of xi");
    check(worst_c < 1e-12, "DG correction divergence = l(+-1)/w");

    /* one 2D element [0.5, 1.5] x [2, 2.25], no neighbours */
    const double x0[2] = {0.5, 2.0}, jac[4] = {0.5, 0.0, 0.0, 0.125};
    const int32_t nbr[4] = {-1, -1, -1, -1};
    pcpf_mesh m;
    memset(&m, 0, sizeof m);
    m.ndims = 2;
    m.order = P;
    m.nelem = 1;
    m.nodes = nodes; m.weights = w; m.deriv = D; m.lminus = lm; m.lplus = lp;
    m.cminus = cm; m.cplus = cp; m.vinv = vinv;
    m.x0 = x0; m.jac = jac; m.nbr = nbr;
    double xs[N * N * 2];
    check(pcpf_solution_coords(&m, xs) == PCPF_OK, "solution coordinates");
    double worst_x = 0.0;
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            const double* x = &xs[(j * N + i) * 2];   /* first index fastest */
            worst_x = fmax(worst_x, fabs(x[0] - (0.5 + 0.5 * (nodes[i] + 1.0))));
            worst_x = fmax(worst_x, fabs(x[1] - (2.0 + 0.125 * (nodes[j] + 1.0))));
        }
    check(worst_x < 1e-15, "affine map of the nodes");

    pcpf_params prm;
    memset(&prm, 0, sizeof prm);
    prm.gamma = 0.09; prm.eps = 1e-3; prm.eps_w = 1e-2; prm.tau = 0.1; prm.nu_max = 1e-3;
    prm.s0 = -5.0; prm.kappa = 5.0; prm.dtau = 1e-3; prm.delta_n = 1e-12;
    prm.delta_g = 1e-12; prm.delta_phi = 1e-12; prm.vel_amp = 1.0; prm.vel_period = 1.0;
    prm.vel_kind = PCPF_VEL_UNIFORM; prm.reset_every = 1000; prm.precond_iters = 10;
    prm.precision = PCPF_FP64;
    size_t nb = 0;
    check(pcpf_workspace_bytes(&m, &prm, &nb) == PCPF_OK && nb >= 5 * 2 * N * N * 8,
          "workspace size");
    prm.kappa = 0.0;
    check(pcpf_workspace_bytes(&m, &prm, &nb) == PCPF_EINVAL &&
              strlen(pcpf_last_error(NULL)) > 0,
          "invalid parameters refused with a message");
    return fails;
}
