/* The C ABI of include/pcpf.h used from plain C99 (host calls only: no GPU needed).
 * Checks the 1D operators of the Gauss-Legendre element against facts of the element
 * (weights sum to the reference length, the derivative of a constant is 0 and of xi is 1,
 * the end interpolations reproduce xi at +-1, the DG correction divergences equal
 * l(+-1)/w), the solution coordinates of an affine box element, the workspace size query
 * and the error path; then the order-2 triangle operators against facts of the triangle
 * (weights sum to the area 1/2, interpolation and derivatives exact on r and s, the
 * lifting's weighted column sums are the edge quadrature weights, whose total is the
 * perimeter 2 + sqrt 2) and the dense description of a one-cell periodic split mesh (two
 * triangles) accepted, and refused with two owners on a pair. Prints one line per check
 * and returns the number of failures. */
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
    prm.kappa = 5.0;

    /* the order-2 triangle */
    enum { TP = 2, TN = TP + 1, TU = (TP + 1) * (TP + 2) / 2, TF = 3 * TN };
    double upt[TU * 2], fpt[TF * 2], M0[TF * TU], TD[2 * TU * TU], LN[2 * TU * TF];
    double L[TU * TF], TV[TU * TU], TW[TU], NH[TF * 2];
    uint8_t top[TU];
    check(pcpf_triangle_operators(TP, upt, fpt, M0, TD, LN, L, TV, top, TW, NH) == PCPF_OK,
          "triangle operators");
    double area = 0.0, wi = 0.0, wd = 0.0, perim = 0.0;
    int ntop = 0;
    for (int i = 0; i < TU; ++i) {
        area += TW[i];
        ntop += top[i] != 0;
        for (int k = 0; k < 2; ++k) {
            double dr = 0.0, ds = 0.0;
            for (int b = 0; b < TU; ++b) {
                dr += TD[(k * TU + i) * TU + b] * upt[2 * b];
                ds += TD[(k * TU + i) * TU + b] * upt[2 * b + 1];
            }
            wd = fmax(wd, fabs(dr - (k == 0)) + fabs(ds - (k == 1)));
        }
    }
    for (int f = 0; f < TF; ++f) {
        double r = 0.0, sv = 0.0, col = 0.0;
        for (int b = 0; b < TU; ++b) {
            r += M0[f * TU + b] * upt[2 * b];
            sv += M0[f * TU + b] * upt[2 * b + 1];
            col += TW[b] * L[b * TF + f];
        }
        wi = fmax(wi, fabs(r - fpt[2 * f]) + fabs(sv - fpt[2 * f + 1]));
        perim += col;
    }
    check(fabs(area - 0.5) < 1e-14 && ntop == TP + 1, "triangle weights and top modes");
    check(wi < 1e-14 && wd < 1e-13, "triangle interpolation and derivatives exact on r, s");
    check(fabs(perim - (2.0 + sqrt(2.0))) < 1e-12, "triangle lifting: edge weights");

    /* one periodic cell of [0, 1]^2 split along its diagonal: A = (c00, c10, c11),
     * B = (c00, c11, c01); A's edges 0, 1, 2 (bottom, right, diagonal) meet B's edges 1
     * (top, across the period), 2 (left, across the period) and 0 (diagonal), each walked
     * the other way */
    const double tjac[2][4] = {{1.0, 1.0, 0.0, 1.0}, {1.0, 0.0, 1.0, 1.0}};
    const double tjinv[2][4] = {{1.0, -1.0, 0.0, 1.0}, {1.0, 0.0, -1.0, 1.0}};
    const double tdet[2] = {1.0, 1.0}, txo[4] = {0.0, 0.0, 0.0, 0.0};
    const int pair_edge[2][3] = {{1, 2, 0}, {2, 0, 1}};
    double tfn[2 * TF * 2], tfs[2 * TF];
    int32_t slot[2 * TF];
    uint8_t own[2 * TF];
    for (int e = 0; e < 2; ++e)
        for (int f = 0; f < TF; ++f) {
            const int edge = f / TN, t = f % TN;
            double nr[2];
            for (int i = 0; i < 2; ++i)
                nr[i] = tjinv[e][0 * 2 + i] * NH[2 * f] + tjinv[e][1 * 2 + i] * NH[2 * f + 1];
            const double mag = sqrt(nr[0] * nr[0] + nr[1] * nr[1]);
            tfn[(e * TF + f) * 2] = nr[0] / mag;
            tfn[(e * TF + f) * 2 + 1] = nr[1] / mag;
            tfs[e * TF + f] = tdet[e] * mag;
            slot[e * TF + f] = (1 - e) * TF + pair_edge[e][edge] * TN + (TN - 1 - t);
            own[e * TF + f] = (nr[0] + nr[1] / sqrt(2.0)) > 0.0;
        }
    pcpf_dense_mesh dm;
    memset(&dm, 0, sizeof dm);
    dm.ndims = 2; dm.order = TP; dm.shape = PCPF_SHAPE_TRIANGLE; dm.nupts = TU; dm.nfpts = TF;
    dm.nelem = 2;
    dm.M0 = M0; dm.D = TD; dm.LiftN = LN; dm.Lift = L; dm.Vinv = TV; dm.topmask = top;
    dm.W = TW; dm.ref_fnorm = NH; dm.jinv = &tjinv[0][0]; dm.detj = tdet; dm.fnorm = tfn;
    dm.fscale = tfs; dm.xorig = txo; dm.jac = &tjac[0][0]; dm.nbr_slot = slot; dm.owner = own;
    dm.period[0] = dm.period[1] = 1.0;
    check(pcpf_workspace_bytes_dense(&dm, &prm, &nb) == PCPF_OK && nb >= 5 * 2 * 2 * TU * 8,
          "dense triangle description accepted");
    own[slot[0]] = own[0];
    check(pcpf_workspace_bytes_dense(&dm, &prm, &nb) == PCPF_EINVAL &&
              strlen(pcpf_last_error(NULL)) > 0,
          "two owners on a flux-point pair refused");
    return fails;
}
