// C-ABI of the FR-PCPF library: validation, workspace layout, the step loop, and the host
// builders of the 1D Gauss-Legendre element.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "pcpf_adjoint.h"
#include "pcpf_internal.h"
#include "pcpf_tri.h"

using namespace pcpf;

namespace {

thread_local std::string g_err = "no error";

pcpf_status fail(std::string* dst, pcpf_status st, const std::string& msg) {
    if (dst) *dst = msg;
    g_err = msg;
    return st;
}

// Status of an entry point that caught an exception (a failed host allocation: every
// other failure is reported by status). The message fits the strings' inline buffer, so
// setting it allocates nothing.
pcpf_status out_of_memory(pcpf_ctx* c) noexcept;

// ------------------------------------------------------------------------------------
// 1D Gauss-Legendre element (host, float64)
// ------------------------------------------------------------------------------------
// Legendre P_n and P_n' by the three-term recurrence.
void legendre(int n, double x, double* p, double* dp) {
    double p0 = 1.0, p1 = x;
    if (n == 0) {
        *p = 1.0;
        *dp = 0.0;
        return;
    }
    for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    *p = p1;
    *dp = n * (x * p1 - p0) / (x * x - 1.0);
}

// Gauss-Legendre nodes (ascending) and weights by Newton iteration on P_n.
void gauss_legendre(int n, double* x, double* w) {
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(n, z, &p, &dp);
            const double dz = p / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        double p, dp;
        legendre(n, z, &p, &dp);
        const double wi = 2.0 / ((1.0 - z * z) * dp * dp);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = wi;
        w[n - 1 - i] = wi;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

// ------------------------------------------------------------------------------------
// triangle element (host, float64): the reference triangle {r, s >= 0, r + s <= 1},
// vertices (0, 0), (1, 0), (0, 1), edges v0 -> v1, v1 -> v2, v2 -> v0
// ------------------------------------------------------------------------------------
// The triangle operators are built in long double (64-bit mantissa on the host) and
// rounded once: the nodal mass matrix of the lattice points is ill conditioned (double
// loses about 1e-11 of the lifting at p = 4 through it).
using LD = long double;

// Legendre P_n and P_n' valid on all of [-1, 1] (P'_k = x P'_{k-1} + k P_{k-1}).
void legendre_pd(int n, LD x, LD* p, LD* dp) {
    if (n == 0) {
        *p = 1.0L;
        *dp = 0.0L;
        return;
    }
    LD p0 = 1.0L, p1 = x, d1 = 1.0L;
    for (int k = 2; k <= n; ++k) {
        const LD p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
        const LD d2 = x * d1 + k * p1;
        p0 = p1;
        p1 = p2;
        d1 = d2;
    }
    *p = p1;
    *dp = d1;
}

// Gauss-Legendre nodes (ascending) and weights in long double: Newton from the double ones.
void gauss_legendre_ld(int n, LD* x, LD* w) {
    std::vector<double> xd(n), wd(n);
    gauss_legendre(n, xd.data(), wd.data());
    for (int i = 0; i < n; ++i) {
        LD z = xd[i], p, dp;
        for (int it = 0; it < 4; ++it) {
            legendre_pd(n, z, &p, &dp);
            z -= p / dp;
        }
        legendre_pd(n, z, &p, &dp);
        x[i] = z;
        w[i] = 2.0L / ((1.0L - z * z) * dp * dp);
    }
}

// The graded basis of P_p used to build the nodal operators: P_a(2r - 1) P_b(2s - 1) for
// a + b = 0, 1, ..., p (b ascending within a degree), with its derivatives.
void tri_basis(int p, LD r, LD s, LD* phi, LD* dr, LD* ds) {
    int m = 0;
    for (int deg = 0; deg <= p; ++deg)
        for (int b = 0; b <= deg; ++b) {
            const int a = deg - b;
            LD pa, dpa, pb, dpb;
            legendre_pd(a, 2.0L * r - 1.0L, &pa, &dpa);
            legendre_pd(b, 2.0L * s - 1.0L, &pb, &dpb);
            phi[m] = pa * pb;
            if (dr) dr[m] = 2.0L * dpa * pb;
            if (ds) ds[m] = 2.0L * pa * dpb;
            ++m;
        }
}

// X = A^-1 B for A n x n, B n x m (row-major), Gauss elimination with partial pivoting.
bool solve_dense(int n, std::vector<LD> A, int m, std::vector<LD>& B) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (!(std::fabs(A[piv * n + c]) > 0.0L)) return false;
        if (piv != c) {
            for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
            for (int k = 0; k < m; ++k) std::swap(B[c * m + k], B[piv * m + k]);
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const LD f = A[r * n + c] / A[c * n + c];
            if (f == 0.0L) continue;
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            for (int k = 0; k < m; ++k) B[r * m + k] -= f * B[c * m + k];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int k = 0; k < m; ++k) B[r * m + k] /= A[r * n + r];
    return true;
}

struct TriOps {
    int p = 0, nu = 0, nf = 0;
    std::vector<double> upt, fpt, nh, wf, M0, D0, D1, Lift, Vinv, W, DH0, DH1;
    std::vector<uint8_t> top;
};

// The order-p triangle of §3.1 with the reading of its solution points (the interior
// lattice ((i + 1/3), (j + 1/3)) / (p + 1), j outer, i inner), Gauss-Legendre flux points on
// each edge in the edge's direction, and DG correction functions: Lift = M^-1 E with the mass
// matrix M = int l_i l_j (by a collapsed Gauss rule, exact for the degree-2p products) and
// E[i][f] = w_f l_i(x_f). The modal transform of the sensor takes the orthonormal basis of
// the graded basis above (Cholesky of its Gram matrix); its degree-p modes are the top ones.
bool tri_operators(int p, TriOps* T) {
    const int n = p + 1, nu = (p + 1) * (p + 2) / 2, nf = 3 * n;
    T->p = p;
    T->nu = nu;
    T->nf = nf;
    std::vector<LD> upt(2 * nu), fpt(2 * nf), nh(2 * nf), wf(nf);
    int i = 0;
    for (int j = 0; j <= p; ++j)
        for (int a = 0; a <= p - j; ++a, ++i) {
            upt[2 * i] = (a + 1.0L / 3.0L) / (p + 1);
            upt[2 * i + 1] = (j + 1.0L / 3.0L) / (p + 1);
        }
    std::vector<LD> xg(n), wg(n);
    gauss_legendre_ld(n, xg.data(), wg.data());
    const LD vx[3] = {0.0L, 1.0L, 0.0L}, vy[3] = {0.0L, 0.0L, 1.0L};
    for (int e = 0; e < 3; ++e) {
        const int a = e, b = (e + 1) % 3;
        const LD tx = vx[b] - vx[a], ty = vy[b] - vy[a];
        const LD L = std::sqrt(tx * tx + ty * ty);
        for (int t = 0; t < n; ++t) {
            const int f = e * n + t;
            fpt[2 * f] = vx[a] + 0.5L * (1.0L + xg[t]) * tx;
            fpt[2 * f + 1] = vy[a] + 0.5L * (1.0L + xg[t]) * ty;
            nh[2 * f] = ty / L;           // outward for the counter-clockwise walk
            nh[2 * f + 1] = -tx / L;
            wf[f] = 0.5L * L * wg[t];
        }
    }
    // Vandermonde V[i][m] = phi_m(x_i); the nodal operators are (basis values) V^-1
    std::vector<LD> V(nu * nu), Vr(nu * nu), Vs(nu * nu), Vf(nf * nu);
    for (int q = 0; q < nu; ++q)
        tri_basis(p, upt[2 * q], upt[2 * q + 1], &V[q * nu], &Vr[q * nu], &Vs[q * nu]);
    for (int f = 0; f < nf; ++f) tri_basis(p, fpt[2 * f], fpt[2 * f + 1], &Vf[f * nu], nullptr, nullptr);
    std::vector<LD> Vi(nu * nu, 0.0L);
    for (int q = 0; q < nu; ++q) Vi[q * nu + q] = 1.0L;
    if (!solve_dense(nu, V, nu, Vi)) return false;
    auto matmul = [](int r, int k, int c, const LD* A, const LD* B, LD* C) {
        for (int x = 0; x < r; ++x)
            for (int y = 0; y < c; ++y) {
                LD acc = 0.0L;
                for (int z = 0; z < k; ++z) acc += A[x * k + z] * B[z * c + y];
                C[x * c + y] = acc;
            }
    };
    std::vector<LD> M0(nf * nu), D0(nu * nu), D1(nu * nu);
    matmul(nf, nu, nu, Vf.data(), Vi.data(), M0.data());
    matmul(nu, nu, nu, Vr.data(), Vi.data(), D0.data());
    matmul(nu, nu, nu, Vs.data(), Vi.data(), D1.data());
    // Gram matrix of the basis and its integrals by the collapsed rule: (u, v) in [0, 1]^2 ->
    // (u, v (1 - u)), Jacobian 1 - u, p + 2 Gauss points each way (exact for degree 2p)
    const int nq = p + 2;
    std::vector<LD> xq(nq), wq(nq), ph(nu);
    gauss_legendre_ld(nq, xq.data(), wq.data());
    std::vector<LD> Gm(nu * nu, 0.0L), gi(nu, 0.0L);
    for (int a = 0; a < nq; ++a)
        for (int b = 0; b < nq; ++b) {
            const LD u = 0.5L * (xq[a] + 1.0L), v = 0.5L * (xq[b] + 1.0L);
            const LD w = 0.25L * wq[a] * wq[b] * (1.0L - u);
            tri_basis(p, u, v * (1.0L - u), ph.data(), nullptr, nullptr);
            for (int x = 0; x < nu; ++x) {
                gi[x] += w * ph[x];
                for (int y = 0; y < nu; ++y) Gm[x * nu + y] += w * ph[x] * ph[y];
            }
        }
    // nodal mass matrix M = V^-T G V^-1 and weights W = V^-T g
    std::vector<LD> ViT(nu * nu), tmp(nu * nu), Mn(nu * nu), W(nu);
    for (int x = 0; x < nu; ++x)
        for (int y = 0; y < nu; ++y) ViT[x * nu + y] = Vi[y * nu + x];
    matmul(nu, nu, nu, ViT.data(), Gm.data(), tmp.data());
    matmul(nu, nu, nu, tmp.data(), Vi.data(), Mn.data());
    matmul(nu, nu, 1, ViT.data(), gi.data(), W.data());
    // Lift = M^-1 E, E[i][f] = w_f M0[f][i]
    std::vector<LD> Em(nu * nf);
    for (int x = 0; x < nu; ++x)
        for (int f = 0; f < nf; ++f) Em[x * nf + f] = wf[f] * M0[f * nu + x];
    if (!solve_dense(nu, Mn, nf, Em)) return false;
    // the volume operators of Step 6 with the lifting of the interpolated normal flux folded
    // in: DH_k = D_k - Lift diag(nhat_k) M0, so that the volume part is DH_0 f~_0 + DH_1 f~_1
    std::vector<LD> DH0(D0), DH1(D1);
    for (int x = 0; x < nu; ++x)
        for (int y = 0; y < nu; ++y)
            for (int f = 0; f < nf; ++f) {
                const LD t = Em[x * nf + f] * M0[f * nu + y];
                DH0[x * nu + y] -= t * nh[2 * f];
                DH1[x * nu + y] -= t * nh[2 * f + 1];
            }
    // orthonormal modes psi = L^-1 phi (G = L L^T): Vinv = L^T V^-1
    std::vector<LD> Lc(nu * nu, 0.0L);
    for (int x = 0; x < nu; ++x)
        for (int y = 0; y <= x; ++y) {
            LD acc = Gm[x * nu + y];
            for (int z = 0; z < y; ++z) acc -= Lc[x * nu + z] * Lc[y * nu + z];
            if (x == y) {
                if (!(acc > 0.0L)) return false;
                Lc[x * nu + x] = std::sqrt(acc);
            } else {
                Lc[x * nu + y] = acc / Lc[y * nu + y];
            }
        }
    std::vector<LD> LT(nu * nu), Vinv(nu * nu);
    for (int x = 0; x < nu; ++x)
        for (int y = 0; y < nu; ++y) LT[x * nu + y] = Lc[y * nu + x];
    matmul(nu, nu, nu, LT.data(), Vi.data(), Vinv.data());
    auto rd = [](const std::vector<LD>& v) { return std::vector<double>(v.begin(), v.end()); };
    T->upt = rd(upt);
    T->fpt = rd(fpt);
    T->nh = rd(nh);
    T->wf = rd(wf);
    T->M0 = rd(M0);
    T->D0 = rd(D0);
    T->D1 = rd(D1);
    T->Lift = rd(Em);
    T->Vinv = rd(Vinv);
    T->W = rd(W);
    T->DH0 = rd(DH0);
    T->DH1 = rd(DH1);
    T->top.resize(nu);
    int m = 0;
    for (int deg = 0; deg <= p; ++deg)
        for (int b = 0; b <= deg; ++b, ++m) T->top[m] = deg == p ? 1 : 0;
    return true;
}

}  // namespace

extern "C" {

int pcpf_abi_version(void) { return PCPF_ABI_VERSION; }

pcpf_status pcpf_line_operators(int32_t order, double* nodes, double* weights, double* deriv,
                                double* lminus, double* lplus, double* cminus, double* cplus,
                                double* vinv) try {
    if (order < 1 || order > PCPF_MAX_ORDER)
        return fail(nullptr, PCPF_EINVAL, "pcpf_line_operators: order out of range");
    if (!nodes || !weights || !deriv || !lminus || !lplus || !cminus || !cplus || !vinv)
        return fail(nullptr, PCPF_EINVAL, "pcpf_line_operators: null output");
    const int n = order + 1;
    gauss_legendre(n, nodes, weights);
    // barycentric weights lambda_b = 1 / prod_{c != b} (xi_b - xi_c)
    std::vector<double> lam(n);
    for (int b = 0; b < n; ++b) {
        double pr = 1.0;
        for (int c = 0; c < n; ++c)
            if (c != b) pr *= nodes[b] - nodes[c];
        lam[b] = 1.0 / pr;
    }
    // derivative matrix of the Lagrange basis at the nodes (barycentric form)
    for (int a = 0; a < n; ++a) {
        double diag = 0.0;
        for (int b = 0; b < n; ++b) {
            if (a == b) continue;
            const double v = (lam[b] / lam[a]) / (nodes[a] - nodes[b]);
            deriv[a * n + b] = v;
            diag -= v;
        }
        deriv[a * n + a] = diag;
    }
    // end values l_b(+-1) (barycentric interpolation)
    for (int s = 0; s < 2; ++s) {
        const double xe = s ? 1.0 : -1.0;
        double den = 0.0;
        for (int c = 0; c < n; ++c) den += lam[c] / (xe - nodes[c]);
        double* out = s ? lplus : lminus;
        for (int b = 0; b < n; ++b) out[b] = (lam[b] / (xe - nodes[b])) / den;
    }
    // DG correction functions: their derivatives at Gauss-Legendre nodes are l(+-1)/w
    for (int a = 0; a < n; ++a) {
        cminus[a] = lminus[a] / weights[a];
        cplus[a] = lplus[a] / weights[a];
    }
    // modal coefficients of the orthonormal Legendre basis: Gauss-Legendre quadrature is
    // exact for the degree-2p products, so chi_j = sum_a w_a Psi_j(xi_a) u_a
    for (int j = 0; j < n; ++j) {
        for (int a = 0; a < n; ++a) {
            double p, dp;
            legendre(j, nodes[a], &p, &dp);
            vinv[j * n + a] = weights[a] * std::sqrt((2.0 * j + 1.0) / 2.0) * p;
        }
    }
    return PCPF_OK;
} catch (...) {
    return out_of_memory(nullptr);
}

pcpf_status pcpf_triangle_operators(int32_t order, double* upt_ref, double* fpt_ref,
                                    double* M0, double* D, double* LiftN, double* Lift,
                                    double* Vinv, uint8_t* topmask, double* W,
                                    double* ref_fnorm) try {
    if (order < 1 || order > TRI_MAX_ORDER)
        return fail(nullptr, PCPF_EINVAL, "pcpf_triangle_operators: order out of range 1..5");
    if (!upt_ref || !fpt_ref || !M0 || !D || !LiftN || !Lift || !Vinv || !topmask || !W || !ref_fnorm)
        return fail(nullptr, PCPF_EINVAL, "pcpf_triangle_operators: null output");
    TriOps T;
    if (!tri_operators(order, &T))
        return fail(nullptr, PCPF_EINVAL, "pcpf_triangle_operators: singular construction");
    const int nu = T.nu, nf = T.nf;
    std::copy(T.upt.begin(), T.upt.end(), upt_ref);
    std::copy(T.fpt.begin(), T.fpt.end(), fpt_ref);
    std::copy(T.M0.begin(), T.M0.end(), M0);
    std::copy(T.D0.begin(), T.D0.end(), D);
    std::copy(T.D1.begin(), T.D1.end(), D + nu * nu);
    std::copy(T.Lift.begin(), T.Lift.end(), Lift);
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < nu; ++i)
            for (int f = 0; f < nf; ++f)
                LiftN[(k * nu + i) * nf + f] = T.Lift[i * nf + f] * T.nh[2 * f + k];
    std::copy(T.Vinv.begin(), T.Vinv.end(), Vinv);
    std::copy(T.top.begin(), T.top.end(), topmask);
    std::copy(T.W.begin(), T.W.end(), W);
    std::copy(T.nh.begin(), T.nh.end(), ref_fnorm);
    return PCPF_OK;
} catch (...) {
    return out_of_memory(nullptr);
}

}  // extern "C"

namespace {

struct MeshInfo {
    int d, p, n, nu, nfa;
    int64_t E;
    int shape = PCPF_SHAPE_TENSOR;
    int nf = 0;    // flux points per element
    int ntr = 0;   // trace slots per element: the + faces (tensor, pushed by the neighbours)
                   // or every flux point (triangle, written by the element itself)
};

pcpf_status check_mesh(const pcpf_mesh* m, MeshInfo* mi, std::string* err) {
    if (!m) return fail(err, PCPF_EINVAL, "mesh is NULL");
    if (m->ndims != 2 && m->ndims != 3) return fail(err, PCPF_EINVAL, "ndims must be 2 or 3");
    const int pmax = m->ndims == 2 ? PCPF_MAX_ORDER : 5;
    if (m->order < 1 || m->order > PCPF_MAX_ORDER)
        return fail(err, PCPF_EINVAL, "order out of range 1..6");
    if (m->order > pmax) return fail(err, PCPF_EUNSUPPORTED, "3D orders above 5 are not built");
    if (m->nelem < 1) return fail(err, PCPF_EINVAL, "nelem must be >= 1");
    if (m->nelem > (int64_t)1 << 31) return fail(err, PCPF_EINVAL, "nelem above 2^31");
    if (!m->nodes || !m->weights || !m->deriv || !m->lminus || !m->lplus || !m->cminus ||
        !m->cplus || !m->vinv || !m->x0 || !m->jac || !m->nbr)
        return fail(err, PCPF_EINVAL, "mesh has a NULL array");
    mi->d = m->ndims;
    mi->p = m->order;
    mi->n = m->order + 1;
    mi->nu = ipow(mi->n, mi->d);
    mi->nfa = ipow(mi->n, mi->d - 1);
    mi->nf = 2 * mi->d * mi->nfa;
    mi->ntr = mi->d * mi->nfa;
    mi->E = m->nelem;
    // the kernels address every per-element array with 32-bit byte offsets
    const int64_t geo = mi->d + 2 * mi->d * mi->d + 1;
    const int64_t per = std::max<int64_t>({mi->nu, geo, 2 * (int64_t)mi->d * mi->nfa});
    if (mi->E * per * 8 >= ((int64_t)1 << 32))
        return fail(err, PCPF_EUNSUPPORTED,
                    "mesh too large: every per-element array must stay below 4 GiB");
    return PCPF_OK;
}

void inv_det(int d, const double* J, double* Ji, double* det) {
    if (d == 2) {
        const double dt = J[0] * J[3] - J[1] * J[2];
        Ji[0] = J[3] / dt;
        Ji[1] = -J[1] / dt;
        Ji[2] = -J[2] / dt;
        Ji[3] = J[0] / dt;
        *det = dt;
    } else {
        const double a = J[0], b = J[1], c = J[2], dd = J[3], e = J[4], f = J[5], g = J[6],
                     h = J[7], i = J[8];
        const double A = e * i - f * h, B = -(dd * i - f * g), C = dd * h - e * g;
        const double dt = a * A + b * B + c * C;
        Ji[0] = A / dt;
        Ji[1] = -(b * i - c * h) / dt;
        Ji[2] = (b * f - c * e) / dt;
        Ji[3] = B / dt;
        Ji[4] = (a * i - c * g) / dt;
        Ji[5] = -(a * f - c * dd) / dt;
        Ji[6] = C / dt;
        Ji[7] = -(a * h - b * g) / dt;
        Ji[8] = (a * e - b * dd) / dt;
        *det = dt;
    }
}

// Physical coordinates of point ref (reference coords) of element e.
void map_point(int d, const double* x0, const double* J, const double* ref, double* x) {
    for (int i = 0; i < d; ++i) {
        double acc = x0[i];
        for (int j = 0; j < d; ++j) acc += J[i * d + j] * (ref[j] + 1.0);
        x[i] = acc;
    }
}

// Reciprocal adjacency, det J > 0, and paired face points equal up to one translation.
pcpf_status check_geometry(const pcpf_mesh* m, const MeshInfo& mi, std::string* err) {
    const int d = mi.d, n = mi.n, nfa = mi.nfa;
    const int64_t E = mi.E;
    std::vector<double> ji(d * d);
    double hmin = 1e300;
    for (int64_t e = 0; e < E; ++e) {
        double det;
        inv_det(d, m->jac + e * d * d, ji.data(), &det);
        if (!(det > 0.0)) return fail(err, PCPF_EINVAL, "element with det J <= 0");
        hmin = std::min(hmin, std::pow(det, 1.0 / d));
        for (int f = 0; f < 2 * d; ++f) {
            const int32_t en = m->nbr[e * 2 * d + f];
            if (en < -1 || en >= E) return fail(err, PCPF_EINVAL, "nbr index out of range");
            if (en >= 0 && m->nbr[(int64_t)en * 2 * d + (f ^ 1)] != e)
                return fail(err, PCPF_EINVAL, "adjacency is not reciprocal (face 2k+1 of e must "
                                              "meet face 2k of nbr[e][2k+1])");
        }
    }
    const double tol = 1e-8 * hmin;
    std::vector<double> ra(d), rb(d), xa(d), xb(d);
    for (int q = 0; q < d; ++q)
        if (!(m->period[q] >= 0.0)) return fail(err, PCPF_EINVAL, "period must be >= 0");
    for (int64_t e = 0; e < E; ++e) {
        for (int k = 0; k < d; ++k) {
            const int32_t en = m->nbr[e * 2 * d + 2 * k + 1];
            if (en < 0) continue;
            for (int t = 0; t < nfa; ++t) {
                int tt = t;
                for (int q = 0; q < d; ++q) {
                    if (q == k) {
                        ra[q] = 1.0;
                        rb[q] = -1.0;
                    } else {
                        ra[q] = rb[q] = m->nodes[tt % n];
                        tt /= n;
                    }
                }
                map_point(d, m->x0 + e * d, m->jac + e * d * d, ra.data(), xa.data());
                map_point(d, m->x0 + (int64_t)en * d, m->jac + (int64_t)en * d * d, rb.data(),
                          xb.data());
                for (int q = 0; q < d; ++q) {
                    double dq = xb[q] - xa[q];
                    if (m->period[q] > 0.0) dq -= std::round(dq / m->period[q]) * m->period[q];
                    if (std::fabs(dq) > tol)
                        return fail(err, PCPF_EINVAL,
                                    "face points of neighbouring elements do not coincide "
                                    "(up to the periods)");
                }
            }
        }
    }
    return PCPF_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    size_t un, us, acc, P, Fp, Tp, sgn, geo, vtab, det64, w64, nbr, ops, flag, partial, red, res;
    size_t total;
};

Layout layout(const MeshInfo& mi, int precision) {
    const size_t r = precision != PCPF_FP64 ? 4 : 8;
    const size_t E = (size_t)mi.E;
    const size_t state = 2 * E * mi.nu * r;              // two variables
    const bool tri = mi.shape == PCPF_SHAPE_TRIANGLE;
    const int geo = mi.d + 2 * mi.d * mi.d + 1;
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.un = take(state);
    L.us = take(state);
    L.acc = take(state);
    L.P = take(state);
    // common fluxes, per variable E N_f slots: tensor [2D][E][NFA] (+ face fluxes, then
    // boundary - face fluxes), triangle [E][N_f]
    L.Fp = take(2 * E * mi.nf * r);
    // traces, per variable E ntr: tensor [D][E][NFA] (pushed), triangle [E][N_f] (own)
    L.Tp = take(2 * E * mi.ntr * r);
    L.sgn = take(E * mi.nu * r);
    L.geo = take(E * geo * r);
    L.vtab = take(tri ? 0 : E * mi.d * (mi.n + 2) * 2 * r);   // velocity tables (axis-aligned)
    L.det64 = take(E * 8);
    L.w64 = take((tri ? mi.nu : mi.n) * 8);
    L.nbr = take(E * (tri ? mi.nf : 2 * mi.d) * 4);
    L.ops = take((tri ? tri_ops_size(mi.p) : ops_size(mi.n)) * r);
    L.flag = take(4);
    L.partial = take(REDUCE_BLOCKS * 8);
    L.red = take(8);
    L.res = take(state);   // scratch residual / sensor output of the residual entry point
    L.total = off;
    return L;
}

}  // namespace

// ------------------------------------------------------------------------------------
// context
// ------------------------------------------------------------------------------------
struct pcpf_ctx {
    MeshInfo mi;
    pcpf_params prm;
    int device = -1;     // the GPU that was current at pcpf_create
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    Layout L;
    Launchers<double> L64;
    Launchers<float> L32;
    double t = 0.0;
    int64_t step = 0;
    bool has_state = false, has_psi = false, has_sign = false;
    bool trace_ok[2] = {false, false};
    bool axis = false;     // every element axis-aligned (diagonal J)
    bool bnd_minus = false;  // some - face (face 2k) has no neighbour
    // checkpointed forward run recorded by pcpf_forward_ckpt (read by pcpf_adjoint)
    bool ck_valid = false, ck_has_psi0 = false;
    int64_t ck_step0 = 0, ck_nsteps = 0, ck_every = 1;
    double ck_amp = 0.0;
    double ck_t0 = 0.0, ck_dt = 0.0;
    // storage hooks of the checkpointed recompute (null outside it)
    void* pc_store_psi0_v = nullptr;
    std::vector<void*> pc_store_stage_v;
    bool pc_reset_hit = false;
    // the last preconditioning: iterations run, final stop-rule RMS (NaN: not computed)
    int32_t pc_iters = -1;
    double pc_rms = 0.0;
    AdjLaunchers<double> A64;
    AdjLaunchers<float> A32;
    std::string err = "no error";
    // per-launch event timing (pcpf_set_timing)
    bool timing = false;
    std::vector<hipEvent_t> events;
    std::vector<int> ev_kind;
    size_t ev_used = 0;
    double kt_ms[PCPF_KT_COUNT] = {0, 0, 0, 0};
    int64_t kt_n[PCPF_KT_COUNT] = {0, 0, 0, 0};
    ~pcpf_ctx() {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
    }
};

namespace {

template <typename R>
struct Ctx {
    pcpf_ctx* c;
    R* plane(size_t off, int v) const {
        return reinterpret_cast<R*>(c->ws + off) + (size_t)v * c->mi.E * c->mi.nu;
    }
    // variable v of the trace buffer
    R* fplane(size_t off, int v) const {
        return reinterpret_cast<R*>(c->ws + off) + (size_t)v * c->mi.E * c->mi.ntr;
    }
    // variable v of the common-flux buffer (E N_f slots per variable)
    R* flux(int v) const {
        return reinterpret_cast<R*>(c->ws + c->L.Fp) + (size_t)v * c->mi.E * c->mi.nf;
    }
    template <typename T>
    T* at(size_t off) const {
        return reinterpret_cast<T*>(c->ws + off);
    }
    const Launchers<R>& Lk() const;
};
template <>
const Launchers<double>& Ctx<double>::Lk() const { return c->L64; }
template <>
const Launchers<float>& Ctx<float>::Lk() const { return c->L32; }

pcpf_status hip_check(pcpf_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return PCPF_OK;
    std::string msg = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c ? &c->err : nullptr, PCPF_EDEVICE, msg);
}

#define HIPCHK(ctx, call)                                          \
    do {                                                           \
        pcpf_status _s = hip_check((ctx), (call), #call);          \
        if (_s != PCPF_OK) return _s;                              \
    } while (0)

double time_factor(const pcpf_params& p, double t) {
    if (p.vel_kind == PCPF_VEL_SINGLE_VORTEX || p.vel_kind == PCPF_VEL_LEVEQUE3D)
        return std::cos(M_PI * t / p.vel_period);
    return 1.0;
}

template <typename R>
Phys<R> phys(const pcpf_params& p, double t) {
    Phys<R> ph;
    ph.gamma = (R)p.gamma;
    ph.eps = (R)p.eps;
    ph.tau = (R)p.tau;
    ph.delta_n = (R)p.delta_n;
    ph.delta_g = (R)p.delta_g;
    ph.nu_max = (R)p.nu_max;
    ph.s0 = (R)p.s0;
    ph.kappa = (R)p.kappa;
    ph.ampg = (R)(p.vel_amp * time_factor(p, t));
    for (int k = 0; k < 3; ++k) ph.u0[k] = (R)p.vel_u0[k];
    ph.vel_kind = p.vel_kind;
    return ph;
}

template <typename R>
GFArgs<R> gf_args(const Ctx<R>& C, const R* u0, const R* u1, double t) {
    pcpf_ctx* c = C.c;
    GFArgs<R> a{};
    a.u[0] = u0;
    a.u[1] = u1;
    for (int v = 0; v < 2; ++v) {
        a.P[v] = C.plane(c->L.P, v);
        a.Fp[v] = C.flux(v);
        a.Tp[v] = C.fplane(c->L.Tp, v);
    }
    a.geo = C.template at<R>(c->L.geo);
    a.nbr = C.template at<int32_t>(c->L.nbr);
    a.ops = C.template at<R>(c->L.ops);
    a.sgn = C.template at<R>(c->L.sgn);
    a.vtab = C.template at<R>(c->L.vtab);
    a.out = nullptr;
    a.E = c->mi.E;
    a.ph = phys<R>(c->prm, t);
    a.axis = c->axis ? 1 : 0;
    a.mf = c->prm.precision == PCPF_BF16 ? 1 : 0;
    a.nphi = c->prm.normal_mode == PCPF_NORMAL_PHI ? 1 : 0;
    a.sgn_current = c->prm.sgn_mode == PCPF_SGN_CURRENT ? 1 : 0;
    a.bnd_minus = c->bnd_minus ? 1 : 0;
    return a;
}

// select the psi plane (index 1) of every two-variable buffer for the one-variable modes
template <typename R>
void psi_only(GFArgs<R>& a) {
    a.u[0] = a.u[1];
    a.P[0] = a.P[1];
    a.Fp[0] = a.Fp[1];
    a.Tp[0] = a.Tp[1];
}

template <typename R>
UPArgs<R> up_args(const Ctx<R>& C) {
    pcpf_ctx* c = C.c;
    UPArgs<R> a{};
    for (int v = 0; v < 2; ++v) {
        a.P[v] = C.plane(c->L.P, v);
        a.Fp[v] = C.flux(v);
        a.un[v] = C.plane(c->L.un, v);
        a.uo[v] = nullptr;
        a.acc[v] = C.plane(c->L.acc, v);
        a.us[v] = C.plane(c->L.us, v);
        a.res[v] = nullptr;
        a.Tp[v] = C.fplane(c->L.Tp, v);
    }
    a.geo = C.template at<R>(c->L.geo);
    a.nbr = C.template at<int32_t>(c->L.nbr);
    a.ops = C.template at<R>(c->L.ops);
    a.flag = C.template at<int>(c->L.flag);
    a.E = c->mi.E;
    a.mf = c->prm.precision == PCPF_BF16 ? 1 : 0;
    return a;
}

template <typename R>
void up_psi_only(UPArgs<R>& a) {
    a.P[0] = a.P[1];
    a.Fp[0] = a.Fp[1];
    a.un[0] = a.un[1];
    a.acc[0] = a.acc[1];
    a.us[0] = a.us[1];
    a.Tp[0] = a.Tp[1];
}

template <typename R>
pcpf_status launch_status(pcpf_ctx* c) {
    return hip_check(c, hipGetLastError(), "kernel launch");
}

// Run launch(ev0, ev1): with timing on, the dispatch records the two events at kernel start
// and end (hipExtLaunchKernelGGL), so their difference is the kernel's execution time.
template <typename F>
pcpf_status timed(pcpf_ctx* c, int kind, F&& launch) {
    if (!c->timing) {
        launch(nullptr, nullptr);
        return PCPF_OK;
    }
    while (c->events.size() < c->ev_used + 2) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e));
        c->events.push_back(e);
    }
    launch(c->events[c->ev_used], c->events[c->ev_used + 1]);
    c->ev_kind.push_back(kind);
    c->ev_used += 2;
    return PCPF_OK;
}

// Accumulate the recorded event pairs (the stream must have been synchronised).
pcpf_status collect_times(pcpf_ctx* c) {
    for (size_t i = 0; i < c->ev_kind.size(); ++i) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->events[2 * i], c->events[2 * i + 1]));
        c->kt_ms[c->ev_kind[i]] += ms;
        c->kt_n[c->ev_kind[i]] += 1;
    }
    c->ev_kind.clear();
    c->ev_used = 0;
    return PCPF_OK;
}

#define TIMED(c, kind, stmt)                                               \
    do {                                                                   \
        pcpf_status _t = timed((c), (kind), [&](hipEvent_t ev0_, hipEvent_t ev1_) { stmt; }); \
        if (_t != PCPF_OK) return _t;                                      \
    } while (0)

// - face traces of the stored state for the variables whose traces are stale
template <typename R>
pcpf_status refresh_traces(const Ctx<R>& C) {
    pcpf_ctx* c = C.c;
    if (c->trace_ok[0] && c->trace_ok[1]) return PCPF_OK;
    TRArgs<R> a{};
    int nv = 0;
    for (int v = 0; v < 2; ++v) {
        if (c->trace_ok[v]) continue;
        a.u[nv] = C.plane(c->L.un, v);
        a.Tp[nv] = C.fplane(c->L.Tp, v);
        ++nv;
    }
    a.ops = C.template at<R>(c->L.ops);
    a.nbr = C.template at<int32_t>(c->L.nbr);
    a.E = c->mi.E;
    C.Lk().trace(nv, a, c->stream);
    c->trace_ok[0] = c->trace_ok[1] = true;
    return launch_status<R>(c);
}

// classic RK4 stage constants
constexpr double RK_B[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
constexpr double RK_C[4] = {0.0, 0.5, 0.5, 1.0};

// Reset + iters pseudo-time RK4 iterations of psi. With store_psi0 / store_stage set (the
// checkpointed recompute of the adjoint), psi0 and the input of every pseudo stage are kept:
// store_stage[4*k + s] receives the psi input of stage s of iteration k.
template <typename R>
pcpf_status reduce_impl(const Ctx<R>& C, int what, const void* d_field, const void* d_ref,
                        double* out);

template <typename R>
pcpf_status precondition_impl(const Ctx<R>& C, int iters, R* store_psi0 = nullptr,
                              R* const* store_stage = nullptr) {
    pcpf_ctx* c = C.c;
    const int64_t n = c->mi.E * c->mi.nu;
    const size_t bytes = (size_t)n * sizeof(R);
    R* phi = C.plane(c->L.un, 0);
    R* psi = C.plane(c->L.un, 1);
    launch_reset<R>(phi, psi, n, c->prm.reset_mode, c->prm.eps_w, c->prm.delta_phi, c->stream);
    if (store_psi0)
        HIPCHK(c, hipMemcpyAsync(store_psi0, psi, bytes, hipMemcpyDeviceToDevice, c->stream));
    // traces of psi0
    {
        TRArgs<R> a{};
        a.u[0] = psi;
        a.Tp[0] = C.fplane(c->L.Tp, 1);
        a.nbr = C.template at<int32_t>(c->L.nbr);
        a.ops = C.template at<R>(c->L.ops);
        a.E = c->mi.E;
        C.Lk().trace(1, a, c->stream);
    }
    // smeared sign; under PCPF_SGN_CURRENT the stages form it from psi0 and their own
    // gradient, so psi0 is kept in its place
    if (c->prm.sgn_mode == PCPF_SGN_CURRENT) {
        HIPCHK(c, hipMemcpyAsync(C.template at<R>(c->L.sgn), psi, bytes,
                                 hipMemcpyDeviceToDevice, c->stream));
    } else {
        GFArgs<R> a = gf_args<R>(C, phi, psi, c->t);
        psi_only(a);
        a.out = C.template at<R>(c->L.sgn);
        C.Lk().grad_flux(GF_SIGN, 1, a, c->stream, nullptr, nullptr);
    }
    c->has_sign = true;
    c->has_psi = true;
    c->pc_iters = 0;
    c->pc_rms = std::numeric_limits<double>::quiet_NaN();
    const double dtau = c->prm.dtau;
    const bool rms_stop = c->prm.stop_mode == PCPF_STOP_RMS;
    R* prev = C.plane(c->L.res, 0);          // psi^(k-1) for the stop rule
    for (int it = 0; it < iters; ++it) {
        if (rms_stop)
            HIPCHK(c, hipMemcpyAsync(prev, psi, bytes, hipMemcpyDeviceToDevice, c->stream));
        if (store_stage)
            HIPCHK(c, hipMemcpyAsync(store_stage[4 * it], psi, bytes, hipMemcpyDeviceToDevice,
                                     c->stream));
        for (int s = 0; s < 4; ++s) {
            R* stage_buf = store_stage ? store_stage[4 * it + (s < 3 ? s + 1 : 0)] : nullptr;
            const R* uin = s == 0 ? psi : (store_stage ? store_stage[4 * it + s] : C.plane(c->L.us, 1));
            GFArgs<R> g = gf_args<R>(C, uin, uin, c->t);
            psi_only(g);
            g.u[0] = uin;
            TIMED(c, PCPF_KT_PC_GRAD_FLUX, C.Lk().grad_flux(GF_PRECOND, 1, g, c->stream, ev0_, ev1_));
            UPArgs<R> u = up_args<R>(C);
            up_psi_only(u);
            if (store_stage && s < 3) u.us[0] = stage_buf;
            u.first = s == 0;
            u.last = s == 3;
            u.bcoef = (R)RK_B[s];
            u.ccoef = (R)(s == 3 ? dtau : RK_C[s + 1] * dtau);
            TIMED(c, PCPF_KT_PC_UPDATE, C.Lk().update(UP_RK, 1, u, c->stream, ev0_, ev1_));
        }
        c->pc_iters = it + 1;
        if (rms_stop) {
            double ss = 0.0;
            pcpf_status st = reduce_impl<R>(C, PCPF_REDUCE_RMS, psi, prev, &ss);
            if (st != PCPF_OK) return st;
            c->pc_rms = ss / dtau;
            if (c->pc_rms <= 0.5) break;
        }
    }
    c->trace_ok[1] = true;   // written by the last update (or by the trace of psi0)
    return launch_status<R>(c);
}

// One classic RK4 step of the stored state. With y_store set (the checkpointed recompute),
// the input of stage s is kept in y_store[2*s + v]; y_next, if set, receives u_{n+1} from the
// last stage as well (the stage-0 input of the next recomputed step), and y0_filled says that
// y_store[0..1] was filled that way by the previous step. A reset at this step changes psi
// before stage 0, so then stage 0's input is copied in any case.
template <typename R>
pcpf_status step_one(const Ctx<R>& C, double dt, R* const* y_store, R* const* y_next = nullptr,
                     bool y0_filled = false) {
    pcpf_ctx* c = C.c;
    const int N = c->prm.reset_every;
    bool reset = false;
    if (!c->has_psi || (N > 0 && c->step % N == 0)) {
        reset = true;
        pcpf_status st = precondition_impl<R>(
            C, c->prm.precond_iters, static_cast<R*>(c->pc_store_psi0_v),
            c->pc_store_stage_v.empty() ? nullptr
                                        : reinterpret_cast<R* const*>(c->pc_store_stage_v.data()));
        if (st != PCPF_OK) return st;
        c->pc_reset_hit = true;
    }
    pcpf_status st = refresh_traces<R>(C);
    if (st != PCPF_OK) return st;
    if (y_store && (reset || !y0_filled)) {
        const size_t bytes = (size_t)c->mi.E * c->mi.nu * sizeof(R);
        for (int v = 0; v < 2; ++v)
            HIPCHK(c, hipMemcpyAsync(y_store[v], C.plane(c->L.un, v), bytes,
                                     hipMemcpyDeviceToDevice, c->stream));
    }
    for (int s = 0; s < 4; ++s) {
        const double ts = c->t + RK_C[s] * dt;
        const R* u0 = s == 0 ? C.plane(c->L.un, 0) : (y_store ? y_store[2 * s] : C.plane(c->L.us, 0));
        const R* u1 = s == 0 ? C.plane(c->L.un, 1) : (y_store ? y_store[2 * s + 1] : C.plane(c->L.us, 1));
        GFArgs<R> g = gf_args<R>(C, u0, u1, ts);
        TIMED(c, PCPF_KT_GRAD_FLUX, C.Lk().grad_flux(GF_PHYS, 2, g, c->stream, ev0_, ev1_));
        UPArgs<R> u = up_args<R>(C);
        if (y_store && s < 3) {
            u.us[0] = y_store[2 * (s + 1)];
            u.us[1] = y_store[2 * (s + 1) + 1];
        }
        if (y_next && s == 3) {
            u.uo[0] = y_next[0];
            u.uo[1] = y_next[1];
        }
        u.first = s == 0;
        u.last = s == 3;
        u.bcoef = (R)RK_B[s];
        u.ccoef = (R)(s == 3 ? dt : RK_C[s + 1] * dt);
        TIMED(c, PCPF_KT_UPDATE, C.Lk().update(UP_RK, 2, u, c->stream, ev0_, ev1_));
    }
    c->t += dt;
    c->step += 1;
    return PCPF_OK;
}

template <typename R>
pcpf_status step_impl(const Ctx<R>& C, double dt, int64_t nsteps) {
    pcpf_ctx* c = C.c;
    HIPCHK(c, hipMemsetAsync(C.template at<int>(c->L.flag), 0, sizeof(int), c->stream));
    for (int64_t i = 0; i < nsteps; ++i) {
        pcpf_status st = step_one<R>(C, dt, nullptr);
        if (st != PCPF_OK) return st;
    }
    pcpf_status st = launch_status<R>(c);
    if (st != PCPF_OK) return st;
    int flag = 0;
    HIPCHK(c, hipMemcpyAsync(&flag, C.template at<int>(c->L.flag), sizeof(int),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    st = collect_times(c);
    if (st != PCPF_OK) return st;
    if (flag) return fail(&c->err, PCPF_ENONFINITE, "state became non-finite or |phi| > 10");
    return PCPF_OK;
}

template <typename R>
pcpf_status residual_impl(const Ctx<R>& C, const void* d_phi, const void* d_psi, double t,
                          int mode, void* d_rphi, void* d_rpsi) {
    pcpf_ctx* c = C.c;
    const R* phi = static_cast<const R*>(d_phi);
    const R* psi = static_cast<const R*>(d_psi);
    if (mode == PCPF_MODE_PHYS) {
        TRArgs<R> tr{};
        tr.u[0] = phi;
        tr.u[1] = psi;
        tr.Tp[0] = C.fplane(c->L.Tp, 0);
        tr.Tp[1] = C.fplane(c->L.Tp, 1);
        tr.nbr = C.template at<int32_t>(c->L.nbr);
        tr.ops = C.template at<R>(c->L.ops);
        tr.E = c->mi.E;
        C.Lk().trace(2, tr, c->stream);
        GFArgs<R> g = gf_args<R>(C, phi, psi, t);
        C.Lk().grad_flux(GF_PHYS, 2, g, c->stream, nullptr, nullptr);
        UPArgs<R> u = up_args<R>(C);
        u.res[0] = static_cast<R*>(d_rphi);
        u.res[1] = static_cast<R*>(d_rpsi);
        C.Lk().update(UP_RESID, 2, u, c->stream, nullptr, nullptr);
        c->trace_ok[0] = c->trace_ok[1] = false;
    } else {
        TRArgs<R> tr{};
        tr.u[0] = psi;
        tr.Tp[0] = C.fplane(c->L.Tp, 1);
        tr.nbr = C.template at<int32_t>(c->L.nbr);
        tr.ops = C.template at<R>(c->L.ops);
        tr.E = c->mi.E;
        C.Lk().trace(1, tr, c->stream);
        GFArgs<R> g = gf_args<R>(C, psi, psi, t);
        psi_only(g);
        g.u[0] = psi;
        C.Lk().grad_flux(GF_PRECOND, 1, g, c->stream, nullptr, nullptr);
        UPArgs<R> u = up_args<R>(C);
        up_psi_only(u);
        u.res[0] = static_cast<R*>(d_rpsi);
        C.Lk().update(UP_RESID, 1, u, c->stream, nullptr, nullptr);
        c->trace_ok[1] = false;
    }
    return launch_status<R>(c);
}

template <typename R>
pcpf_status sensor_impl(const Ctx<R>& C, const void* d_psi, void* d_nu) {
    pcpf_ctx* c = C.c;
    GFArgs<R> g = gf_args<R>(C, static_cast<const R*>(d_psi), static_cast<const R*>(d_psi),
                             c->t);
    g.out = static_cast<R*>(d_nu);
    C.Lk().grad_flux(GF_SENSOR, 1, g, c->stream, nullptr, nullptr);
    return launch_status<R>(c);
}

template <typename R>
pcpf_status reduce_impl(const Ctx<R>& C, int what, const void* d_field, const void* d_ref,
                        double* out) {
    pcpf_ctx* c = C.c;
    RDArgs<R> a{};
    a.field = d_field ? static_cast<const R*>(d_field) : C.plane(c->L.un, 0);
    a.ref = static_cast<const R*>(d_ref);
    a.det64 = C.template at<double>(c->L.det64);
    a.w64 = C.template at<double>(c->L.w64);
    a.partial = C.template at<double>(c->L.partial);
    a.E = c->mi.E;
    a.kind = what;
    const int64_t total = c->mi.E * c->mi.nu;
    int nb = (int)std::min<int64_t>(REDUCE_BLOCKS, (total + REDUCE_THREADS - 1) / REDUCE_THREADS);
    if (nb < 1) nb = 1;
    C.Lk().reduce(a, nb, c->stream);
    double* red = C.template at<double>(c->L.red);
    launch_reduce_final(a.partial, nb, red, c->stream);
    pcpf_status st = launch_status<R>(c);
    if (st != PCPF_OK) return st;
    HIPCHK(c, hipMemcpyAsync(out, red, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (what == PCPF_REDUCE_RMS) *out = std::sqrt(*out / (double)total);
    return PCPF_OK;
}

// sin(pi x) on the host: x reduced exactly to [-1, 1], then sin
double sinpi_host(double x) { return std::sin(M_PI * (x - 2.0 * std::nearbyint(0.5 * x))); }

template <typename R>
pcpf_status upload(pcpf_ctx* c, const pcpf_mesh* m) {
    const MeshInfo& mi = c->mi;
    const int d = mi.d, n = mi.n;
    const int G = d + 2 * d * d + 1;
    const int64_t E = mi.E;
    std::vector<R> geo((size_t)E * G);
    std::vector<double> det64(E);
    std::vector<double> ji(d * d);
    for (int64_t e = 0; e < E; ++e) {
        double det;
        const double* J = m->jac + e * d * d;
        inv_det(d, J, ji.data(), &det);
        R* g = geo.data() + e * G;
        for (int k = 0; k < d; ++k) g[k] = (R)m->x0[e * d + k];
        for (int k = 0; k < d * d; ++k) g[d + k] = (R)J[k];
        for (int k = 0; k < d * d; ++k) g[d + d * d + k] = (R)ji[k];
        g[d + 2 * d * d] = (R)det;
        det64[e] = det;
    }
    // operator block: D1, DH = D1 - cp (x) lp + cm (x) lm, VINV, DT = D1 - cp (x) lp, lm, lp,
    // cm, cp, xi, w
    std::vector<R> ops(ops_size(n));
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            const double d1 = m->deriv[a * n + b];
            ops[OP_D1 + a * n + b] = (R)d1;
            ops[op_dh(n) + a * n + b] =
                (R)(d1 - m->cplus[a] * m->lplus[b] + m->cminus[a] * m->lminus[b]);
            ops[op_vinv(n) + a * n + b] = (R)m->vinv[a * n + b];
            ops[op_dt(n) + a * n + b] = (R)(d1 - m->cplus[a] * m->lplus[b]);
        }
    for (int a = 0; a < n; ++a) {
        ops[op_lm(n) + a] = (R)m->lminus[a];
        ops[op_lp(n) + a] = (R)m->lplus[a];
        ops[op_cm(n) + a] = (R)m->cminus[a];
        ops[op_cp(n) + a] = (R)m->cplus[a];
        ops[op_xi(n) + a] = (R)m->nodes[a];
        ops[op_w(n) + a] = (R)m->weights[a];
    }
    // sin^2(pi x_k) and sin(2 pi x_k) at the n nodes and at both ends (xi = -1, +1) of every
    // element axis: the factors of the trigonometric velocity fields on axis-aligned meshes
    // (time-independent)
    const int ntb = n + 2;
    const bool trig = c->prm.vel_kind == PCPF_VEL_SINGLE_VORTEX || c->prm.vel_kind == PCPF_VEL_LEVEQUE3D;
    std::vector<R> vtab(trig ? (size_t)E * d * ntb * 2 : 0);
    for (int64_t e = 0; trig && e < E; ++e)
        for (int k = 0; k < d; ++k)
            for (int j = 0; j < ntb; ++j) {
                const double xr = j < n ? m->nodes[j] : (j == n ? -1.0 : 1.0);
                const double x = m->x0[e * d + k] + m->jac[(e * d + k) * d + k] * (xr + 1.0);
                const size_t o = (((size_t)e * d + k) * ntb + j) * 2;
                const double sx = sinpi_host(x);
                vtab[o] = (R)(sx * sx);
                vtab[o + 1] = (R)sinpi_host(2.0 * x);
            }
    Ctx<R> C{c};
    HIPCHK(c, hipMemcpyAsync(C.template at<R>(c->L.geo), geo.data(), geo.size() * sizeof(R),
                             hipMemcpyHostToDevice, c->stream));
    if (trig)
        HIPCHK(c, hipMemcpyAsync(C.template at<R>(c->L.vtab), vtab.data(), vtab.size() * sizeof(R),
                                 hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(C.template at<double>(c->L.det64), det64.data(), E * 8,
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(C.template at<double>(c->L.w64), m->weights, n * 8,
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(C.template at<int32_t>(c->L.nbr), m->nbr, E * 2 * d * 4,
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(C.template at<R>(c->L.ops), ops.data(), ops.size() * sizeof(R),
                             hipMemcpyHostToDevice, c->stream));
    // face buffers start defined (boundary + face slots of Tp are never written)
    HIPCHK(c, hipMemsetAsync(c->ws + c->L.Fp, 0, c->L.sgn - c->L.Fp, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PCPF_OK;
}

// ------------------------------------------------------------------------------------
// adjoint: checkpointed reverse sweep
// ------------------------------------------------------------------------------------
struct AdjLayout {
    size_t seg, pre0, pre, yb, ya, rb, ub, tb, gp, sb, pb, pa, prb, apart, total;
};

AdjLayout adj_layout(const pcpf_ctx* c, int64_t every) {
    const size_t r = c->prm.precision != PCPF_FP64 ? 4 : 8;
    const size_t S = (size_t)c->mi.E * c->mi.nu;
    const size_t F = (size_t)c->mi.E * c->mi.d * c->mi.nfa;
    const int epb = c->prm.precision != PCPF_FP64 ? c->A32.epb : c->A64.epb;
    const size_t nblocks = (size_t)((c->mi.E + epb - 1) / epb);
    AdjLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.seg = take((size_t)every * 4 * 2 * S * r);
    L.pre0 = take(S * r);
    L.pre = take((size_t)(c->prm.precond_iters > 0 ? c->prm.precond_iters : 1) * 4 * S * r);
    L.yb = take(2 * S * r);
    L.ya = take(2 * S * r);
    L.rb = take(2 * S * r);
    L.ub = take(2 * S * r);
    L.tb = take(2 * F * r);
    L.gp = take(2 * F * r);
    L.sb = take(S * r);
    L.pb = take(S * r);
    L.pa = take(S * r);
    L.prb = take(S * r);
    L.apart = take(nblocks * 8);
    L.total = off;
    return L;
}

template <typename R>
const AdjLaunchers<R>& adj_launchers(const pcpf_ctx* c);
template <>
const AdjLaunchers<double>& adj_launchers<double>(const pcpf_ctx* c) { return c->A64; }
template <>
const AdjLaunchers<float>& adj_launchers<float>(const pcpf_ctx* c) { return c->A32; }

// Reverse-sweep options of one stage: where its push (lifting adjoint and forward traces of
// Y, to the faces' owners) runs, and whether the stage starts a reverse step.
template <typename R>
struct AdjStageOpt {
    bool push = true;                 // launch the push first (false: the previous stage's
                                      // finish has done it)
    const R* const* seed_yb = nullptr;  // start of a reverse step: ya <- yb, R^ = alpha yb
    R* const* seed_ya = nullptr;
    double seed_alpha = 0.0;
    R* const* ynext = nullptr;        // the next stage's input: its push runs at the end of
                                      // this stage's finish (rnext must be set)
};

// One stage of the reverse sweep: Y^ = (dR/dY)^T R^ for the stage input Y (nvar planes);
// then ya += Y^ and rnext = c_prev yb + c_cur Y^ (either may be null).
template <typename R>
pcpf_status adj_stage(const Ctx<R>& C, int mode, R* const* Y, R* const* rb, double t, R* const* ub,
                      R* const* tb, R* const* gp, R* sb, R* const* ya, R* const* rnext,
                      R* const* yb, double c_prev, double c_cur, double* apart,
                      const AdjStageOpt<R>& opt = AdjStageOpt<R>()) {
    pcpf_ctx* c = C.c;
    const int nvar = mode == AD_PHYS ? 2 : 1;
    const AdjLaunchers<R>& AL = adj_launchers<R>(c);
    TRArgs<R> tr{};
    for (int v = 0; v < nvar; ++v) {
        tr.u[v] = Y[v];
        tr.Tp[v] = C.fplane(c->L.Tp, v);
    }
    tr.nbr = C.template at<int32_t>(c->L.nbr);
    tr.ops = C.template at<R>(c->L.ops);
    tr.E = c->mi.E;
    if (mode == AD_SIGN) {
        C.Lk().trace(nvar, tr, c->stream);
    } else if (opt.push) {
        // the lifting-adjoint push also pushes the forward traces of Y
        AJPush<R> p{};
        for (int v = 0; v < nvar; ++v) {
            p.rbar[v] = rb[v];
            p.gp[v] = gp[v];
            p.u[v] = Y[v];
            p.Tp[v] = tr.Tp[v];
            if (opt.seed_yb) {
                p.seed_yb[v] = opt.seed_yb[v];
                p.seed_ya[v] = opt.seed_ya[v];
                p.seed_rb[v] = rb[v];
            }
        }
        p.seed_alpha = (R)opt.seed_alpha;
        p.geo = C.template at<R>(c->L.geo);
        p.nbr = tr.nbr;
        p.ops = tr.ops;
        p.E = c->mi.E;
        AL.push(nvar, p, c->stream);
    }
    AJMain<R> m{};
    for (int v = 0; v < nvar; ++v) {
        m.u[v] = Y[v];
        m.Tp[v] = tr.Tp[v];
        m.rbar[v] = rb ? rb[v] : nullptr;
        m.gp[v] = gp[v];
        m.ub[v] = ub[v];
        m.tb[v] = tb[v];
    }
    m.sb = sb;
    m.sgn = C.template at<R>(c->L.sgn);
    m.geo = C.template at<R>(c->L.geo);
    m.nbr = tr.nbr;
    m.ops = tr.ops;
    m.apart = apart;
    m.E = c->mi.E;
    m.ph = phys<R>(c->prm, t);
    m.amp = (R)c->prm.vel_amp;
    m.gt = (R)time_factor(c->prm, t);
    AL.main(mode, m, c->stream);
    AJFinish<R> f{};
    for (int v = 0; v < nvar; ++v) {
        f.ub[v] = ub[v];
        f.tb[v] = tb[v];
        f.ya[v] = ya ? ya[v] : nullptr;
        f.rnext[v] = rnext ? rnext[v] : nullptr;
        f.yb[v] = yb ? yb[v] : nullptr;
    }
    f.nbr = tr.nbr;
    f.ops = tr.ops;
    f.E = c->mi.E;
    f.c_prev = (R)c_prev;
    f.c_cur = (R)c_cur;
    if (opt.ynext) {
        for (int v = 0; v < nvar; ++v) {
            f.ynext[v] = opt.ynext[v];
            f.gp[v] = gp[v];
            f.Tp[v] = tr.Tp[v];
        }
        f.geo = C.template at<R>(c->L.geo);
    }
    AL.finish(nvar, f, c->stream);
    return launch_status<R>(c);
}

template <typename R>
pcpf_status forward_ckpt_impl(const Ctx<R>& C, double dt, int64_t nsteps, int64_t every,
                              void* d_ckpt) {
    pcpf_ctx* c = C.c;
    const size_t S = (size_t)c->mi.E * c->mi.nu;
    c->ck_valid = false;
    c->ck_step0 = c->step;
    c->ck_t0 = c->t;
    c->ck_dt = dt;
    c->ck_nsteps = nsteps;
    c->ck_every = every;
    c->ck_amp = c->prm.vel_amp;
    c->ck_has_psi0 = c->has_psi;
    HIPCHK(c, hipMemsetAsync(C.template at<int>(c->L.flag), 0, sizeof(int), c->stream));
    R* ck = static_cast<R*>(d_ckpt);
    for (int64_t i = 0; i < nsteps; ++i) {
        if (i % every == 0) {
            // state before step i (before a reset of that step)
            HIPCHK(c, hipMemcpyAsync(ck + (size_t)(i / every) * 2 * S, C.plane(c->L.un, 0),
                                     2 * S * sizeof(R), hipMemcpyDeviceToDevice, c->stream));
        }
        pcpf_status st = step_one<R>(C, dt, nullptr);
        if (st != PCPF_OK) return st;
    }
    pcpf_status st = launch_status<R>(c);
    if (st != PCPF_OK) return st;
    int flag = 0;
    HIPCHK(c, hipMemcpyAsync(&flag, C.template at<int>(c->L.flag), sizeof(int),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    st = collect_times(c);
    if (st != PCPF_OK) return st;
    if (flag) return fail(&c->err, PCPF_ENONFINITE, "state became non-finite or |phi| > 10");
    c->ck_valid = true;
    return PCPF_OK;
}

template <typename R>
pcpf_status adjoint_impl(const Ctx<R>& C, const void* d_ckpt, void* d_scratch,
                         const void* d_gphi, const void* d_gpsi, void* d_gphi0, void* d_gpsi0,
                         double* g_amp) {
    pcpf_ctx* c = C.c;
    const AdjLayout A = adj_layout(c, c->ck_every);
    const size_t S = (size_t)c->mi.E * c->mi.nu;
    const size_t Sb = S * sizeof(R);
    const size_t F = (size_t)c->mi.E * c->mi.d * c->mi.nfa;
    char* w = static_cast<char*>(d_scratch);
    auto at = [&](size_t off) { return reinterpret_cast<R*>(w + off); };
    R* yb[2] = {at(A.yb), at(A.yb) + S};
    R* ya[2] = {at(A.ya), at(A.ya) + S};
    R* rb[2] = {at(A.rb), at(A.rb) + S};
    R* ub[2] = {at(A.ub), at(A.ub) + S};
    R* tb[2] = {at(A.tb), at(A.tb) + F};
    R* gp[2] = {at(A.gp), at(A.gp) + F};
    R* sb = at(A.sb);
    R* pb = at(A.pb);
    R* pa = at(A.pa);
    R* prb = at(A.prb);
    R* pre0 = at(A.pre0);
    double* apart = reinterpret_cast<double*>(w + A.apart);
    const int K = c->prm.precond_iters;
    const double dt = c->ck_dt, dtau = c->prm.dtau;
    const double amp_now = c->prm.vel_amp;
    c->prm.vel_amp = c->ck_amp;   // recompute and differentiate the recorded run
    struct RestoreAmp {
        pcpf_ctx* c;
        double a;
        ~RestoreAmp() { c->prm.vel_amp = a; }
    } restore_amp{c, amp_now};
    const int64_t every = c->ck_every, nsteps = c->ck_nsteps;
    const int64_t nseg = (nsteps + every - 1) / every;
    const R* ck = static_cast<const R*>(d_ckpt);
    // exchange slots that are never written (boundary faces) must read as zero
    HIPCHK(c, hipMemsetAsync(w + A.tb, 0, A.sb - A.tb, c->stream));
    HIPCHK(c, hipMemsetAsync(w + A.apart, 0, A.total - A.apart, c->stream));
    HIPCHK(c, hipMemcpyAsync(yb[0], d_gphi, Sb, hipMemcpyDeviceToDevice, c->stream));
    if (d_gpsi) HIPCHK(c, hipMemcpyAsync(yb[1], d_gpsi, Sb, hipMemcpyDeviceToDevice, c->stream));
    else HIPCHK(c, hipMemsetAsync(yb[1], 0, Sb, c->stream));
    std::vector<R*> pre_stage((size_t)(K > 0 ? K : 1) * 4);
    for (size_t i = 0; i < pre_stage.size(); ++i) pre_stage[i] = at(A.pre) + i * S;
    for (int64_t j = nseg - 1; j >= 0; --j) {
        const int64_t seg_start = j * every;
        const int64_t nloc = std::min(every, nsteps - seg_start);
        // recompute the segment from its checkpoint, keeping every stage input
        HIPCHK(c, hipMemcpyAsync(C.plane(c->L.un, 0), ck + (size_t)j * 2 * S, 2 * Sb,
                                 hipMemcpyDeviceToDevice, c->stream));
        c->has_psi = (j == 0) ? c->ck_has_psi0 : true;
        c->step = c->ck_step0 + seg_start;
        c->t = c->ck_t0 + (double)seg_start * dt;
        c->trace_ok[0] = c->trace_ok[1] = false;
        c->pc_store_psi0_v = pre0;
        c->pc_store_stage_v.assign(pre_stage.begin(), pre_stage.end());
        int64_t reset_local = -1;
        for (int64_t i = 0; i < nloc; ++i) {
            R* ys[8];
            for (int s = 0; s < 4; ++s)
                for (int v = 0; v < 2; ++v) ys[2 * s + v] = at(A.seg) + ((size_t)i * 4 + s) * 2 * S + v * S;
            // the next step's stage-0 slot, written by this step's last stage
            R* yn[2] = {at(A.seg) + (size_t)(i + 1) * 4 * 2 * S, at(A.seg) + (size_t)(i + 1) * 4 * 2 * S + S};
            c->pc_reset_hit = false;
            pcpf_status st = step_one<R>(C, dt, ys, i + 1 < nloc ? yn : nullptr, i > 0);
            if (st != PCPF_OK) return st;
            if (c->pc_reset_hit) {
                if (reset_local >= 0)
                    return fail(&c->err, PCPF_EINVAL, "two resets in one checkpoint segment");
                reset_local = i;
            }
        }
        c->pc_store_psi0_v = nullptr;
        c->pc_store_stage_v.clear();
        // reverse sweep over the segment
        for (int64_t i = nloc - 1; i >= 0; --i) {
            const double tn = c->ck_t0 + (double)(seg_start + i) * dt;
            // stage 4's push also seeds the step (ya <- yb, rb <- dt b_4 yb); each later
            // stage's push runs at the end of the previous stage's finish
            for (int s = 3; s >= 0; --s) {
                R* Y[2] = {at(A.seg) + ((size_t)i * 4 + s) * 2 * S, at(A.seg) + ((size_t)i * 4 + s) * 2 * S + S};
                R* Yn[2] = {nullptr, nullptr};
                if (s > 0) {
                    Yn[0] = at(A.seg) + ((size_t)i * 4 + s - 1) * 2 * S;
                    Yn[1] = Yn[0] + S;
                }
                AdjStageOpt<R> opt;
                opt.push = s == 3;
                if (s == 3) {
                    opt.seed_yb = yb;
                    opt.seed_ya = ya;
                    opt.seed_alpha = dt * RK_B[3];
                }
                opt.ynext = s > 0 ? Yn : nullptr;
                pcpf_status st = adj_stage<R>(C, AD_PHYS, Y, rb, tn + RK_C[s] * dt, ub, tb, gp, nullptr,
                                              ya, s > 0 ? rb : nullptr, yb,
                                              s > 0 ? dt * RK_B[s - 1] : 0.0, s > 0 ? dt * RK_C[s] : 0.0,
                                              apart, opt);
                if (st != PCPF_OK) return st;
            }
            std::swap(yb[0], ya[0]);
            std::swap(yb[1], ya[1]);
            if (i == reset_local) {
                // psi after the preconditioning came from phi_n; the previous psi was discarded
                HIPCHK(c, hipMemcpyAsync(pb, yb[1], Sb, hipMemcpyDeviceToDevice, c->stream));
                HIPCHK(c, hipMemsetAsync(yb[1], 0, Sb, c->stream));
                HIPCHK(c, hipMemsetAsync(sb, 0, Sb, c->stream));
                R* pbv[1] = {pb};
                for (int k = K - 1; k >= 0; --k) {
                    R* pav[1] = {pa};
                    R* prv[1] = {prb};
                    R* ubv[1] = {ub[0]};
                    R* tbv[1] = {tb[0]};
                    R* gpv[1] = {gp[0]};
                    pbv[0] = pb;
                    for (int s = 3; s >= 0; --s) {
                        R* Y[1] = {pre_stage[(size_t)k * 4 + s]};
                        R* Yn[1] = {s > 0 ? pre_stage[(size_t)k * 4 + s - 1] : nullptr};
                        AdjStageOpt<R> opt;
                        opt.push = s == 3;
                        if (s == 3) {
                            opt.seed_yb = pbv;
                            opt.seed_ya = pav;
                            opt.seed_alpha = dtau * RK_B[3];
                        }
                        opt.ynext = s > 0 ? Yn : nullptr;
                        pcpf_status st = adj_stage<R>(C, AD_PRECOND, Y, prv, c->t, ubv, tbv, gpv, sb, pav,
                                                      s > 0 ? prv : nullptr, pbv,
                                                      s > 0 ? dtau * RK_B[s - 1] : 0.0,
                                                      s > 0 ? dtau * RK_C[s] : 0.0, apart, opt);
                        if (st != PCPF_OK) return st;
                    }
                    std::swap(pb, pa);
                }
                // sign VJP: psi0^ += d sgn / d psi0 ^T sb
                {
                    R* Y[1] = {pre0};
                    R* ubv[1] = {ub[0]};
                    R* tbv[1] = {tb[0]};
                    R* gpv[1] = {gp[0]};
                    R* accv[1] = {pb};
                    pcpf_status st = adj_stage<R>(C, AD_SIGN, Y, nullptr, c->t, ubv, tbv, gpv, sb, accv,
                                                  nullptr, nullptr, 0.0, 0.0, apart);
                    if (st != PCPF_OK) return st;
                }
                // reset VJP into phi_n^ (phi_n is the stage-0 input of step n)
                const R* phin = at(A.seg) + (size_t)i * 4 * 2 * S;
                launch_reset_adj<R>(yb[0], pb, phin, (int64_t)S, c->prm.reset_mode, c->prm.eps_w,
                                    c->prm.delta_phi, c->stream);
                pcpf_status st = launch_status<R>(c);
                if (st != PCPF_OK) return st;
            }
        }
    }
    HIPCHK(c, hipMemcpyAsync(d_gphi0, yb[0], Sb, hipMemcpyDeviceToDevice, c->stream));
    if (d_gpsi0) HIPCHK(c, hipMemcpyAsync(d_gpsi0, yb[1], Sb, hipMemcpyDeviceToDevice, c->stream));
    const int epb = adj_launchers<R>(c).epb;
    const int nb = (int)((c->mi.E + epb - 1) / epb);
    double* red = C.template at<double>(c->L.red);
    launch_reduce_final(apart, nb, red, c->stream);
    pcpf_status st = launch_status<R>(c);
    if (st != PCPF_OK) return st;
    double ga = 0.0;
    HIPCHK(c, hipMemcpyAsync(&ga, red, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (g_amp) *g_amp = ga;
    c->has_state = false;   // the stored state was used as the recompute register
    return PCPF_OK;
}

pcpf_status check_ctx(pcpf_ctx* c) {
    if (!c) return fail(nullptr, PCPF_EINVAL, "ctx is NULL");
    return PCPF_OK;
}

#define DISPATCH(c, fn, ...) \
    ((c)->prm.precision != PCPF_FP64 ? fn<float>(Ctx<float>{c}, __VA_ARGS__) \
                                     : fn<double>(Ctx<double>{c}, __VA_ARGS__))

pcpf_status check_params(const pcpf_params* p, std::string* err) {
    if (!p) return fail(err, PCPF_EINVAL, "params is NULL");
    if (p->precision != PCPF_FP64 && p->precision != PCPF_FP32 && p->precision != PCPF_BF16)
        return fail(err, PCPF_EUNSUPPORTED, "precision must be PCPF_FP64, PCPF_FP32 or PCPF_BF16");
    if (p->vel_kind < 0 || p->vel_kind > 3) return fail(err, PCPF_EINVAL, "unknown vel_kind");
    if (p->reset_mode != PCPF_RESET_LINEAR && p->reset_mode != PCPF_RESET_LOGIT)
        return fail(err, PCPF_EINVAL, "unknown reset_mode");
    if (p->reset_every < 0 || p->precond_iters < 0)
        return fail(err, PCPF_EINVAL, "reset_every and precond_iters must be >= 0");
    if (!(p->gamma >= 0) || !(p->eps >= 0) || !(p->tau >= 0) || !(p->nu_max >= 0) ||
        !(p->kappa > 0) || !(p->delta_n > 0) || !(p->delta_g > 0) || !(p->delta_phi > 0) ||
        !(p->delta_phi < 0.5) || !std::isfinite(p->s0) || !std::isfinite(p->vel_amp) ||
        !std::isfinite(p->dtau))
        return fail(err, PCPF_EINVAL, "parameter out of range");
    if ((p->vel_kind == PCPF_VEL_SINGLE_VORTEX || p->vel_kind == PCPF_VEL_LEVEQUE3D) &&
        !(p->vel_period > 0))
        return fail(err, PCPF_EINVAL, "vel_period must be > 0");
    if (p->reset_mode == PCPF_RESET_LOGIT && !(p->eps_w > 0))
        return fail(err, PCPF_EINVAL, "eps_w must be > 0 for the LOGIT reset");
    if (p->normal_mode != PCPF_NORMAL_PSI && p->normal_mode != PCPF_NORMAL_PHI)
        return fail(err, PCPF_EINVAL, "unknown normal_mode");
    if (p->sgn_mode != PCPF_SGN_PSI0 && p->sgn_mode != PCPF_SGN_CURRENT)
        return fail(err, PCPF_EINVAL, "unknown sgn_mode");
    if (p->stop_mode != PCPF_STOP_FIXED && p->stop_mode != PCPF_STOP_RMS)
        return fail(err, PCPF_EINVAL, "unknown stop_mode");
    return PCPF_OK;
}

pcpf_status out_of_memory(pcpf_ctx* c) noexcept {
    static const char kMsg[] = "out of memory";
    if (c) c->err = kMsg;
    g_err = kMsg;
    return PCPF_ENOMEM;
}

// ------------------------------------------------------------------------------------
// dense description -> line factors
// ------------------------------------------------------------------------------------
// The dense operators of a Gauss-Legendre tensor element are Kronecker products of the 1D
// factors with identities (interpolation and lifting touch one line; derivatives act
// along one axis), so such a description is mapped onto the 1D factors the kernels apply.
struct DenseLine {
    std::vector<double> nodes, weights, deriv, lm, lp, cm, cp, vinv, x0, jac;
    std::vector<int32_t> nbr;
    pcpf_mesh m{};
};

// Compare a given operator with the expected one entry by entry (relative to the largest
// expected entry, at least 1).
template <typename F>
bool same_operator(const double* given, size_t count, F expected) {
    double scale = 1.0;
    for (size_t i = 0; i < count; ++i) scale = std::max(scale, std::fabs(expected(i)));
    for (size_t i = 0; i < count; ++i)
        if (!(std::fabs(given[i] - expected(i)) <= 1e-12 * scale)) return false;
    return true;
}

pcpf_status dense_to_line(const pcpf_dense_mesh* dm, DenseLine* h) {
    if (!dm) return fail(nullptr, PCPF_EINVAL, "dense mesh is NULL");
    if (dm->ndims != 2 && dm->ndims != 3) return fail(nullptr, PCPF_EINVAL, "ndims must be 2 or 3");
    if (dm->shape != PCPF_SHAPE_TENSOR) return fail(nullptr, PCPF_EINVAL, "unknown element shape");
    const int d = dm->ndims, p = dm->order;
    const int pmax = d == 2 ? PCPF_MAX_ORDER : 5;
    if (p < 1 || p > PCPF_MAX_ORDER) return fail(nullptr, PCPF_EINVAL, "order out of range 1..6");
    if (p > pmax) return fail(nullptr, PCPF_EUNSUPPORTED, "3D orders above 5 are not built");
    const int n = p + 1, nu = ipow(n, d), nfa = ipow(n, d - 1), nf = 2 * d * nfa;
    if (dm->nupts != nu || dm->nfpts != nf)
        return fail(nullptr, PCPF_EINVAL, "nupts / nfpts do not match the tensor element of order p");
    if (dm->nelem < 1 || dm->nelem > ((int64_t)1 << 31))
        return fail(nullptr, PCPF_EINVAL, "nelem out of range");
    if (!dm->M0 || !dm->D || !dm->LiftN || !dm->Lift || !dm->Vinv || !dm->topmask || !dm->W ||
        !dm->ref_fnorm || !dm->jinv || !dm->detj || !dm->fnorm || !dm->fscale || !dm->xorig ||
        !dm->nbr_slot || !dm->owner)
        return fail(nullptr, PCPF_EINVAL, "dense mesh has a NULL array");
    const int64_t E = dm->nelem;
    h->nodes.resize(n);
    h->weights.resize(n);
    h->deriv.resize(n * n);
    h->lm.resize(n);
    h->lp.resize(n);
    h->cm.resize(n);
    h->cp.resize(n);
    h->vinv.resize(n * n);
    pcpf_status st = pcpf_line_operators(p, h->nodes.data(), h->weights.data(), h->deriv.data(),
                                         h->lm.data(), h->lp.data(), h->cm.data(), h->cp.data(),
                                         h->vinv.data());
    if (st != PCPF_OK) return st;
    // multi-indices of the solution points and the (face, direction, side, tangential
    // position) of the flux points
    std::vector<int> mi((size_t)nu * d), fk(nf), fs(nf), tmi((size_t)nf * d, -1);
    for (int i = 0; i < nu; ++i) {
        int r = i;
        for (int k = 0; k < d; ++k) {
            mi[(size_t)i * d + k] = r % n;
            r /= n;
        }
    }
    for (int j = 0; j < nf; ++j) {
        const int f = j / nfa, k = f / 2;
        int t = j % nfa;
        fk[j] = k;
        fs[j] = f % 2;
        for (int m = 0; m < d; ++m) {
            if (m == k) continue;
            tmi[(size_t)j * d + m] = t % n;
            t /= n;
        }
    }
    // point i lies on the line through flux point j (every index but the normal one agrees)
    auto on_line = [&](int i, int j) {
        for (int m = 0; m < d; ++m)
            if (m != fk[j] && mi[(size_t)i * d + m] != tmi[(size_t)j * d + m]) return false;
        return true;
    };
    auto lift1 = [&](int i, int j) {
        if (!on_line(i, j)) return 0.0;
        return (fs[j] ? h->cp : h->cm)[mi[(size_t)i * d + fk[j]]];
    };
    const char* bad = nullptr;
    if (!same_operator(dm->M0, (size_t)nf * nu, [&](size_t q) {
            const int j = (int)(q / nu), i = (int)(q % nu);
            return on_line(i, j) ? (fs[j] ? h->lp : h->lm)[mi[(size_t)i * d + fk[j]]] : 0.0;
        }))
        bad = "M0";
    else if (!same_operator(dm->D, (size_t)d * nu * nu, [&](size_t q) {
                 const int k = (int)(q / ((size_t)nu * nu));
                 const int i = (int)((q / nu) % nu), i2 = (int)(q % nu);
                 for (int m = 0; m < d; ++m)
                     if (m != k && mi[(size_t)i * d + m] != mi[(size_t)i2 * d + m]) return 0.0;
                 return h->deriv[mi[(size_t)i * d + k] * n + mi[(size_t)i2 * d + k]];
             }))
        bad = "D";
    else if (!same_operator(dm->Lift, (size_t)nu * nf, [&](size_t q) {
                 return lift1((int)(q / nf), (int)(q % nf));
             }))
        bad = "Lift";
    else if (!same_operator(dm->LiftN, (size_t)d * nu * nf, [&](size_t q) {
                 const int k = (int)(q / ((size_t)nu * nf));
                 const int i = (int)((q / nf) % nu), j = (int)(q % nf);
                 if (fk[j] != k) return 0.0;
                 return (fs[j] ? 1.0 : -1.0) * lift1(i, j);
             }))
        bad = "LiftN";
    else if (!same_operator(dm->Vinv, (size_t)nu * nu, [&](size_t q) {
                 const int J = (int)(q / nu), i = (int)(q % nu);
                 double v = 1.0;
                 for (int k = 0; k < d; ++k)
                     v *= h->vinv[mi[(size_t)J * d + k] * n + mi[(size_t)i * d + k]];
                 return v;
             }))
        bad = "Vinv";
    else if (!same_operator(dm->W, (size_t)nu, [&](size_t i) {
                 double w = 1.0;
                 for (int k = 0; k < d; ++k) w *= h->weights[mi[i * d + k]];
                 return w;
             }))
        bad = "W";
    else if (!same_operator(dm->ref_fnorm, (size_t)nf * d, [&](size_t q) {
                 const int j = (int)(q / d), k = (int)(q % d);
                 return k == fk[j] ? (fs[j] ? 1.0 : -1.0) : 0.0;
             }))
        bad = "ref_fnorm";
    if (bad)
        return fail(nullptr, PCPF_EUNSUPPORTED,
                    std::string("dense operator ") + bad +
                        " is not that of the Gauss-Legendre tensor element with DG correction "
                        "functions in the stated point and face order (the only element built)");
    for (int J = 0; J < nu; ++J) {
        int top = 0;
        for (int k = 0; k < d; ++k) top |= mi[(size_t)J * d + k] == p;
        if ((dm->topmask[J] != 0) != (top != 0))
            return fail(nullptr, PCPF_EUNSUPPORTED,
                        "topmask does not select the modes of degree p in some direction");
    }
    // geometry: one affine map per element
    h->x0.assign(dm->xorig, dm->xorig + E * d);
    h->jac.resize((size_t)E * d * d);
    std::vector<double> Jm(d * d), Ji(d * d);
    for (int64_t e = 0; e < E; ++e) {
        const double* gi = dm->jinv + e * d * d;
        double det;
        if (dm->jac) {
            std::copy(dm->jac + e * d * d, dm->jac + (e + 1) * d * d, Jm.begin());
            inv_det(d, Jm.data(), Ji.data(), &det);
            double sc = 0.0;
            for (int q = 0; q < d * d; ++q) sc = std::max(sc, std::fabs(gi[q]));
            for (int q = 0; q < d * d; ++q)
                if (!(std::fabs(Ji[q] - gi[q]) <= 1e-12 * sc))
                    return fail(nullptr, PCPF_EINVAL, "jinv is not the inverse of jac");
        } else {
            double idet;
            inv_det(d, gi, Jm.data(), &idet);
            det = 1.0 / idet;
        }
        if (!(det > 0.0)) return fail(nullptr, PCPF_EINVAL, "element with det J <= 0");
        if (!(std::fabs(det - dm->detj[e]) <= 1e-12 * det))
            return fail(nullptr, PCPF_EINVAL, "detj disagrees with the Jacobian");
        for (int j = 0; j < nf; ++j) {
            const int k = fk[j];
            const double sg = fs[j] ? 1.0 : -1.0;
            double mag = 0.0;
            for (int i = 0; i < d; ++i) mag += gi[k * d + i] * gi[k * d + i];
            mag = std::sqrt(mag);
            for (int i = 0; i < d; ++i)
                if (!(std::fabs(dm->fnorm[(e * nf + j) * d + i] - sg * gi[k * d + i] / mag) <= 1e-12))
                    return fail(nullptr, PCPF_EINVAL, "fnorm disagrees with the Jacobian");
            if (!(std::fabs(dm->fscale[e * nf + j] - det * mag) <= 1e-12 * det * mag))
                return fail(nullptr, PCPF_EINVAL, "fscale disagrees with the Jacobian");
        }
        std::copy(Jm.begin(), Jm.end(), h->jac.begin() + e * d * d);
    }
    // connectivity: whole faces paired with the opposite face of one neighbour
    h->nbr.assign((size_t)E * 2 * d, -1);
    const int64_t S = E * nf;
    for (int64_t e = 0; e < E; ++e) {
        for (int f = 0; f < 2 * d; ++f) {
            const int64_t s0 = e * nf + (int64_t)f * nfa;
            const int32_t first = dm->nbr_slot[s0];
            if (first < -1 || first >= S) return fail(nullptr, PCPF_EINVAL, "nbr_slot out of range");
            const int64_t en = first >= 0 ? first / nf : -1;
            for (int t = 0; t < nfa; ++t) {
                const int64_t sl = s0 + t;
                const int32_t ns = dm->nbr_slot[sl];
                if (ns < -1 || ns >= S) return fail(nullptr, PCPF_EINVAL, "nbr_slot out of range");
                if (ns < 0) {
                    if (first >= 0)
                        return fail(nullptr, PCPF_EUNSUPPORTED,
                                    "a face with paired and boundary flux points is not built");
                    if (dm->owner[sl] != 1)
                        return fail(nullptr, PCPF_EINVAL, "a boundary flux point must be owned");
                    continue;
                }
                if (dm->nbr_slot[ns] != sl)
                    return fail(nullptr, PCPF_EINVAL, "nbr_slot pairs are not reciprocal");
                if ((dm->owner[sl] != 0) == (dm->owner[ns] != 0) || dm->owner[sl] > 1 ||
                    dm->owner[ns] > 1)
                    return fail(nullptr, PCPF_EINVAL, "each flux-point pair needs exactly one owner");
                if (ns / nf != en || ns % nf != (int64_t)(f ^ 1) * nfa + t)
                    return fail(nullptr, PCPF_EUNSUPPORTED,
                                "face pairing other than the whole opposite face with flux points "
                                "in the same tangential order is not built");
                if ((dm->owner[sl] != 0) != ((f & 1) != 0))
                    return fail(nullptr, PCPF_EUNSUPPORTED,
                                "owners other than the + face side (LDG beta = +1/2 there) are "
                                "not built");
            }
            h->nbr[e * 2 * d + f] = (int32_t)en;
        }
    }
    pcpf_mesh& m = h->m;
    m.ndims = d;
    m.order = p;
    m.nelem = E;
    m.nodes = h->nodes.data();
    m.weights = h->weights.data();
    m.deriv = h->deriv.data();
    m.lminus = h->lm.data();
    m.lplus = h->lp.data();
    m.cminus = h->cm.data();
    m.cplus = h->cp.data();
    m.vinv = h->vinv.data();
    m.x0 = h->x0.data();
    m.jac = h->jac.data();
    m.nbr = h->nbr.data();
    for (int q = 0; q < 3; ++q) m.period[q] = dm->period[q];
    return PCPF_OK;
}

}  // namespace

// ------------------------------------------------------------------------------------
// dense description of a triangle mesh
// ------------------------------------------------------------------------------------
struct TriHolder {
    TriOps T;
    int64_t E = 0;
    std::vector<double> x0, jac;
    std::vector<int32_t> code;   // 2 s' + owner, -1 on a boundary
};

pcpf_status dense_to_tri(const pcpf_dense_mesh* dm, TriHolder* h) {
    const int p = dm->order;
    if (dm->ndims != 2) return fail(nullptr, PCPF_EINVAL, "triangles are two-dimensional");
    if (p < 1 || p > TRI_MAX_ORDER) return fail(nullptr, PCPF_EUNSUPPORTED, "triangle orders 1..5 are built");
    const int nu = tri_nupts(p), nf = tri_nfpts(p);
    if (dm->nupts != nu || dm->nfpts != nf)
        return fail(nullptr, PCPF_EINVAL, "nupts / nfpts do not match the triangle of order p");
    const int64_t E = dm->nelem;
    if (E < 1 || E * nf >= ((int64_t)1 << 30)) return fail(nullptr, PCPF_EINVAL, "nelem out of range");
    if (!dm->M0 || !dm->D || !dm->LiftN || !dm->Lift || !dm->Vinv || !dm->topmask || !dm->W ||
        !dm->ref_fnorm || !dm->jinv || !dm->detj || !dm->fnorm || !dm->fscale || !dm->xorig ||
        !dm->nbr_slot || !dm->owner)
        return fail(nullptr, PCPF_EINVAL, "dense mesh has a NULL array");
    TriOps& T = h->T;
    if (!tri_operators(p, &T)) return fail(nullptr, PCPF_EINVAL, "triangle operators: singular construction");
    const char* bad = nullptr;
    if (!same_operator(dm->M0, (size_t)nf * nu, [&](size_t q) { return T.M0[q]; }))
        bad = "M0";
    else if (!same_operator(dm->D, (size_t)2 * nu * nu, [&](size_t q) {
                 return q < (size_t)nu * nu ? T.D0[q] : T.D1[q - (size_t)nu * nu];
             }))
        bad = "D";
    else if (!same_operator(dm->Lift, (size_t)nu * nf, [&](size_t q) { return T.Lift[q]; }))
        bad = "Lift";
    else if (!same_operator(dm->LiftN, (size_t)2 * nu * nf, [&](size_t q) {
                 const size_t k = q / ((size_t)nu * nf), r = q % ((size_t)nu * nf);
                 return T.Lift[r] * T.nh[2 * (r % nf) + k];
             }))
        bad = "LiftN";
    else if (!same_operator(dm->Vinv, (size_t)nu * nu, [&](size_t q) { return T.Vinv[q]; }))
        bad = "Vinv";
    else if (!same_operator(dm->W, (size_t)nu, [&](size_t q) { return T.W[q]; }))
        bad = "W";
    else if (!same_operator(dm->ref_fnorm, (size_t)2 * nf, [&](size_t q) { return T.nh[q]; }))
        bad = "ref_fnorm";
    if (bad)
        return fail(nullptr, PCPF_EUNSUPPORTED,
                    std::string("dense operator ") + bad +
                        " is not that of the library's triangle (interior lattice solution "
                        "points, Gauss-Legendre edge points, DG correction functions)");
    for (int j = 0; j < nu; ++j)
        if ((dm->topmask[j] != 0) != (T.top[j] != 0))
            return fail(nullptr, PCPF_EUNSUPPORTED, "topmask does not select the degree-p modes");
    h->E = E;
    h->x0.assign(dm->xorig, dm->xorig + E * 2);
    h->jac.resize((size_t)E * 4);
    std::vector<double> Jm(4), Ji(4);
    double hmin = 1e300;
    for (int64_t e = 0; e < E; ++e) {
        const double* gi = dm->jinv + e * 4;
        double det;
        if (dm->jac) {
            std::copy(dm->jac + e * 4, dm->jac + (e + 1) * 4, Jm.begin());
            inv_det(2, Jm.data(), Ji.data(), &det);
            double sc = 0.0;
            for (int q = 0; q < 4; ++q) sc = std::max(sc, std::fabs(gi[q]));
            for (int q = 0; q < 4; ++q)
                if (!(std::fabs(Ji[q] - gi[q]) <= 1e-12 * sc))
                    return fail(nullptr, PCPF_EINVAL, "jinv is not the inverse of jac");
        } else {
            double idet;
            inv_det(2, gi, Jm.data(), &idet);
            det = 1.0 / idet;
        }
        if (!(det > 0.0)) return fail(nullptr, PCPF_EINVAL, "element with det J <= 0");
        if (!(std::fabs(det - dm->detj[e]) <= 1e-12 * det))
            return fail(nullptr, PCPF_EINVAL, "detj disagrees with the Jacobian");
        hmin = std::min(hmin, std::sqrt(det));
        for (int f = 0; f < nf; ++f) {
            double nr[2];
            for (int i = 0; i < 2; ++i) nr[i] = gi[0 * 2 + i] * T.nh[2 * f] + gi[1 * 2 + i] * T.nh[2 * f + 1];
            const double mag = std::sqrt(nr[0] * nr[0] + nr[1] * nr[1]);
            for (int i = 0; i < 2; ++i)
                if (!(std::fabs(dm->fnorm[(e * nf + f) * 2 + i] - nr[i] / mag) <= 1e-12))
                    return fail(nullptr, PCPF_EINVAL, "fnorm disagrees with the Jacobian");
            if (!(std::fabs(dm->fscale[e * nf + f] - det * mag) <= 1e-12 * det * mag))
                return fail(nullptr, PCPF_EINVAL, "fscale disagrees with the Jacobian");
        }
        std::copy(Jm.begin(), Jm.end(), h->jac.begin() + e * 4);
    }
    // pairing: reciprocal, one owner per pair, coincident points up to the periods
    const int64_t S = E * nf;
    const double tol = 1e-8 * hmin;
    h->code.assign((size_t)S, -1);
    auto point = [&](int64_t sl, double* x) {
        const int64_t e = sl / nf;
        const int f = (int)(sl % nf);
        const double* J = &h->jac[e * 4];
        for (int i = 0; i < 2; ++i)
            x[i] = h->x0[e * 2 + i] + J[i * 2 + 0] * T.fpt[2 * f] + J[i * 2 + 1] * T.fpt[2 * f + 1];
    };
    for (int64_t sl = 0; sl < S; ++sl) {
        const int32_t ns = dm->nbr_slot[sl];
        if (ns < -1 || ns >= S) return fail(nullptr, PCPF_EINVAL, "nbr_slot out of range");
        if (dm->owner[sl] > 1) return fail(nullptr, PCPF_EINVAL, "owner flags must be 0 or 1");
        if (ns < 0) {
            if (dm->owner[sl] != 1) return fail(nullptr, PCPF_EINVAL, "a boundary flux point must be owned");
            continue;
        }
        if (dm->nbr_slot[ns] != sl) return fail(nullptr, PCPF_EINVAL, "nbr_slot pairs are not reciprocal");
        if (dm->owner[sl] + dm->owner[ns] != 1)
            return fail(nullptr, PCPF_EINVAL, "each flux-point pair needs exactly one owner");
        double xa[2], xb[2];
        point(sl, xa);
        point(ns, xb);
        for (int q = 0; q < 2; ++q) {
            double dq = xb[q] - xa[q];
            if (dm->period[q] > 0.0) dq -= std::round(dq / dm->period[q]) * dm->period[q];
            if (std::fabs(dq) > tol)
                return fail(nullptr, PCPF_EINVAL,
                            "paired flux points do not coincide (up to the periods)");
        }
        h->code[sl] = 2 * ns + dm->owner[sl];
    }
    return PCPF_OK;
}

template <typename R>
pcpf_status upload_tri(pcpf_ctx* c, const TriHolder& h) {
    const TriOps& T = h.T;
    const int nu = T.nu, nf = T.nf, G = 11;
    const int64_t E = h.E;
    std::vector<R> geo((size_t)E * G);
    std::vector<double> det64(E), ji(4);
    for (int64_t e = 0; e < E; ++e) {
        double det;
        const double* J = &h.jac[e * 4];
        inv_det(2, J, ji.data(), &det);
        R* g = geo.data() + e * G;
        for (int k = 0; k < 2; ++k) g[k] = (R)h.x0[e * 2 + k];
        for (int k = 0; k < 4; ++k) g[2 + k] = (R)J[k];
        for (int k = 0; k < 4; ++k) g[6 + k] = (R)ji[k];
        g[10] = (R)det;
        det64[e] = det;
    }
    std::vector<R> ops(tri_ops_size(T.p));
    size_t o = 0;
    auto put = [&](const std::vector<double>& v) {
        for (double x : v) ops[o++] = (R)x;
    };
    put(T.M0);
    put(T.D0);
    put(T.D1);
    put(T.Lift);
    put(T.Vinv);
    for (int j = 0; j < nu; ++j) ops[o++] = (R)T.top[j];
    put(T.upt);
    put(T.fpt);
    put(T.nh);
    put(T.DH0);
    put(T.DH1);
    (void)nf;
    Ctx<R> C{c};
    HIPCHK(c, hipMemcpyAsync(C.template at<R>(c->L.geo), geo.data(), geo.size() * sizeof(R),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(C.template at<double>(c->L.det64), det64.data(), E * 8,
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(C.template at<double>(c->L.w64), T.W.data(), nu * 8,
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(C.template at<int32_t>(c->L.nbr), h.code.data(), h.code.size() * 4,
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(C.template at<R>(c->L.ops), ops.data(), ops.size() * sizeof(R),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(c->ws + c->L.Fp, 0, c->L.sgn - c->L.Fp, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PCPF_OK;
}

MeshInfo tri_info(int p, int64_t E) {
    MeshInfo mi{};
    mi.d = 2;
    mi.p = p;
    mi.n = p + 1;
    mi.nu = tri_nupts(p);
    mi.nfa = p + 1;
    mi.E = E;
    mi.shape = PCPF_SHAPE_TRIANGLE;
    mi.nf = tri_nfpts(p);
    mi.ntr = mi.nf;
    return mi;
}

pcpf_status create_tri(const TriHolder& h, const pcpf_params* p, void* d_ws, size_t ws_bytes,
                       void* stream, pcpf_ctx** out) {
    pcpf_status st = check_params(p, nullptr);
    if (st != PCPF_OK) return st;
    if (p->precision == PCPF_BF16)
        return fail(nullptr, PCPF_EUNSUPPORTED, "the BF16 form is built for tensor elements");
    const MeshInfo mi = tri_info(h.T.p, h.E);
    if (mi.E * std::max(mi.nu, mi.nf) * 8 >= ((int64_t)1 << 32))
        return fail(nullptr, PCPF_EUNSUPPORTED, "mesh too large: per-element arrays above 4 GiB");
    Layout L = layout(mi, p->precision);
    if (!d_ws || ws_bytes < L.total)
        return fail(nullptr, PCPF_EINVAL, "workspace missing or smaller than pcpf_workspace_bytes");
    if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0)
        return fail(nullptr, PCPF_EINVAL, "workspace must be 256-byte aligned");
    std::unique_ptr<pcpf_ctx> hold(new pcpf_ctx());
    pcpf_ctx* c = hold.get();
    c->mi = mi;
    c->prm = *p;
    c->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&c->device) != hipSuccess)
        return fail(nullptr, PCPF_EDEVICE, "hipGetDevice failed");
    c->ws = static_cast<char*>(d_ws);
    c->L = L;
    c->axis = false;
    c->bnd_minus = false;
    const bool ok = p->precision != PCPF_FP64 ? get_tri_launchers<float>(mi.p, &c->L32)
                                              : get_tri_launchers<double>(mi.p, &c->L64);
    if (!ok) return fail(nullptr, PCPF_EUNSUPPORTED, "no triangle kernels built for this order");
    st = p->precision != PCPF_FP64 ? upload_tri<float>(c, h) : upload_tri<double>(c, h);
    if (st != PCPF_OK) {
        g_err = c->err;
        return st;
    }
    *out = hold.release();
    return PCPF_OK;
}

// ------------------------------------------------------------------------------------
// static adjoint scratch (pcpf_adjoint_static): one array per GPU the library runs on,
// held until the process ends. In host code `scratch` names a host-side stand-in, not
// device memory: its device address on each GPU comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is passed on.
// ------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[PCPF_ADJOINT_STATIC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's static scratch (the context's device must be current).
pcpf_status static_scratch(pcpf_ctx* c, void** out) {
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev != c->device)
        return fail(&c->err, PCPF_EINVAL, "pcpf_adjoint_static: make the context's GPU current");
    if (dev < 0 || dev >= MAX_DEVICES)
        return fail(&c->err, PCPF_EUNSUPPORTED, "pcpf_adjoint_static: device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(&c->err, PCPF_EDEVICE,
                        std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PCPF_OK;
}

extern "C" {

const char* pcpf_last_error(const pcpf_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_err.c_str();
}

pcpf_status pcpf_solution_coords(const pcpf_mesh* m, double* xs) try {
    MeshInfo mi;
    pcpf_status st = check_mesh(m, &mi, nullptr);
    if (st != PCPF_OK) return st;
    if (!xs) return fail(nullptr, PCPF_EINVAL, "xs is NULL");
    std::vector<double> ref(mi.d);
    for (int64_t e = 0; e < mi.E; ++e)
        for (int i = 0; i < mi.nu; ++i) {
            int r = i;
            for (int k = 0; k < mi.d; ++k) {
                ref[k] = m->nodes[r % mi.n];
                r /= mi.n;
            }
            map_point(mi.d, m->x0 + e * mi.d, m->jac + e * mi.d * mi.d, ref.data(),
                      xs + (e * mi.nu + i) * mi.d);
        }
    return PCPF_OK;
} catch (...) {
    return out_of_memory(nullptr);
}

pcpf_status pcpf_workspace_bytes(const pcpf_mesh* m, const pcpf_params* p, size_t* nbytes) try {
    MeshInfo mi;
    pcpf_status st = check_mesh(m, &mi, nullptr);
    if (st != PCPF_OK) return st;
    st = check_params(p, nullptr);
    if (st != PCPF_OK) return st;
    if (!nbytes) return fail(nullptr, PCPF_EINVAL, "nbytes is NULL");
    *nbytes = layout(mi, p->precision).total;
    return PCPF_OK;
} catch (...) {
    return out_of_memory(nullptr);
}

pcpf_status pcpf_create(const pcpf_mesh* m, const pcpf_params* p, void* d_ws, size_t ws_bytes,
                        void* stream, pcpf_ctx** out) try {
    if (!out) return fail(nullptr, PCPF_EINVAL, "out is NULL");
    *out = nullptr;
    MeshInfo mi;
    pcpf_status st = check_mesh(m, &mi, nullptr);
    if (st != PCPF_OK) return st;
    st = check_params(p, nullptr);
    if (st != PCPF_OK) return st;
    st = check_geometry(m, mi, nullptr);
    if (st != PCPF_OK) return st;
    Layout L = layout(mi, p->precision);
    if (!d_ws || ws_bytes < L.total)
        return fail(nullptr, PCPF_EINVAL, "workspace missing or smaller than pcpf_workspace_bytes");
    if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0)
        return fail(nullptr, PCPF_EINVAL, "workspace must be 256-byte aligned");
    std::unique_ptr<pcpf_ctx> hold(new pcpf_ctx());
    pcpf_ctx* c = hold.get();
    c->mi = mi;
    c->prm = *p;
    c->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&c->device) != hipSuccess)
        return fail(nullptr, PCPF_EDEVICE, "hipGetDevice failed");
    c->ws = static_cast<char*>(d_ws);
    c->L = L;
    c->axis = true;
    for (int64_t e = 0; e < mi.E && c->axis; ++e)
        for (int i = 0; i < mi.d; ++i)
            for (int j = 0; j < mi.d; ++j)
                if (i != j && m->jac[(e * mi.d + i) * mi.d + j] != 0.0) c->axis = false;
    for (int64_t e = 0; e < mi.E && !c->bnd_minus; ++e)
        for (int k = 0; k < mi.d; ++k)
            if (m->nbr[e * 2 * mi.d + 2 * k] < 0) c->bnd_minus = true;
    bool ok = p->precision != PCPF_FP64
                  ? (get_launchers<float>(mi.d, mi.p, &c->L32) && get_adj_launchers<float>(mi.d, mi.p, &c->A32))
                  : (get_launchers<double>(mi.d, mi.p, &c->L64) && get_adj_launchers<double>(mi.d, mi.p, &c->A64));
    if (!ok) return fail(nullptr, PCPF_EUNSUPPORTED, "no kernels built for this (d, p)");
    st = p->precision != PCPF_FP64 ? upload<float>(c, m) : upload<double>(c, m);
    if (st != PCPF_OK) {
        g_err = c->err;
        return st;
    }
    *out = hold.release();
    return PCPF_OK;
} catch (...) {
    return out_of_memory(nullptr);
}

pcpf_status pcpf_workspace_bytes_dense(const pcpf_dense_mesh* dm, const pcpf_params* p,
                                       size_t* nbytes) try {
    if (dm && dm->shape == PCPF_SHAPE_TRIANGLE) {
        TriHolder th;
        pcpf_status st = dense_to_tri(dm, &th);
        if (st != PCPF_OK) return st;
        st = check_params(p, nullptr);
        if (st != PCPF_OK) return st;
        if (p->precision == PCPF_BF16)
            return fail(nullptr, PCPF_EUNSUPPORTED, "the BF16 form is built for tensor elements");
        if (!nbytes) return fail(nullptr, PCPF_EINVAL, "nbytes is NULL");
        *nbytes = layout(tri_info(th.T.p, th.E), p->precision).total;
        return PCPF_OK;
    }
    DenseLine h;
    pcpf_status st = dense_to_line(dm, &h);
    if (st != PCPF_OK) return st;
    return pcpf_workspace_bytes(&h.m, p, nbytes);
} catch (...) {
    return out_of_memory(nullptr);
}

pcpf_status pcpf_create_dense(const pcpf_dense_mesh* dm, const pcpf_params* p, void* d_ws,
                              size_t ws_bytes, void* stream, pcpf_ctx** out) try {
    if (!out) return fail(nullptr, PCPF_EINVAL, "out is NULL");
    *out = nullptr;
    if (dm && dm->shape == PCPF_SHAPE_TRIANGLE) {
        TriHolder th;
        pcpf_status st = dense_to_tri(dm, &th);
        if (st != PCPF_OK) return st;
        return create_tri(th, p, d_ws, ws_bytes, stream, out);
    }
    DenseLine h;
    pcpf_status st = dense_to_line(dm, &h);
    if (st != PCPF_OK) return st;
    return pcpf_create(&h.m, p, d_ws, ws_bytes, stream, out);
} catch (...) {
    return out_of_memory(nullptr);
}

void pcpf_destroy(pcpf_ctx* c) { delete c; }

pcpf_status pcpf_sizes(const pcpf_ctx* c, int64_t* nelem, int32_t* nupts) try {
    if (!c) return fail(nullptr, PCPF_EINVAL, "ctx is NULL");
    if (nelem) *nelem = c->mi.E;
    if (nupts) *nupts = c->mi.nu;
    return PCPF_OK;
} catch (...) {
    return out_of_memory(nullptr);
}

pcpf_status pcpf_set_state(pcpf_ctx* c, const void* d_phi, const void* d_psi, double t,
                           int64_t step) try {
    if (check_ctx(c) != PCPF_OK) return PCPF_EINVAL;
    if (!d_phi) return fail(&c->err, PCPF_EINVAL, "d_phi is NULL");
    if (step < 0) return fail(&c->err, PCPF_EINVAL, "step must be >= 0");
    const size_t bytes = (size_t)c->mi.E * c->mi.nu * (c->prm.precision != PCPF_FP64 ? 4 : 8);
    HIPCHK(c, hipMemcpyAsync(c->ws + c->L.un, d_phi, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (d_psi)
        HIPCHK(c, hipMemcpyAsync(c->ws + c->L.un + bytes, d_psi, bytes, hipMemcpyDeviceToDevice,
                                 c->stream));
    c->t = t;
    c->step = step;
    c->has_state = true;
    c->has_psi = d_psi != nullptr;
    c->trace_ok[0] = c->trace_ok[1] = false;
    return PCPF_OK;
} catch (...) {
    return out_of_memory(c);
}

pcpf_status pcpf_get_state(pcpf_ctx* c, void* d_phi, void* d_psi, double* t, int64_t* step) try {
    if (check_ctx(c) != PCPF_OK) return PCPF_EINVAL;
    if (!c->has_state) return fail(&c->err, PCPF_ESTATE, "no state set");
    const size_t bytes = (size_t)c->mi.E * c->mi.nu * (c->prm.precision != PCPF_FP64 ? 4 : 8);
    if (d_phi)
        HIPCHK(c, hipMemcpyAsync(d_phi, c->ws + c->L.un, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (d_psi) {
        if (!c->has_psi) return fail(&c->err, PCPF_ESTATE, "psi not available before a reset");
        HIPCHK(c, hipMemcpyAsync(d_psi, c->ws + c->L.un + bytes, bytes, hipMemcpyDeviceToDevice,
                                 c->stream));
    }
    if (t) *t = c->t;
    if (step) *step = c->step;
    return PCPF_OK;
} catch (...) {
    return out_of_memory(c);
}

pcpf_status pcpf_step(pcpf_ctx* c, double dt, int64_t nsteps) try {
    if (check_ctx(c) != PCPF_OK) return PCPF_EINVAL;
    if (!c->has_state) return fail(&c->err, PCPF_ESTATE, "no state set");
    if (!std::isfinite(dt) || nsteps < 0) return fail(&c->err, PCPF_EINVAL, "bad dt or nsteps");
    return DISPATCH(c, step_impl, dt, nsteps);
} catch (...) {
    return out_of_memory(c);
}

pcpf_status pcpf_precondition(pcpf_ctx* c, int32_t iters) try {
    if (check_ctx(c) != PCPF_OK) return PCPF_EINVAL;
    if (!c->has_state) return fail(&c->err, PCPF_ESTATE, "no state set");
    const int k = iters < 0 ? c->prm.precond_iters : iters;
    pcpf_status st = DISPATCH(c, precondition_impl, k);
    if (st != PCPF_OK || !c->timing) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return collect_times(c);
} catch (...) {
    return out_of_memory(c);
}

pcpf_status pcpf_precond_info(const pcpf_ctx* c, int32_t* iters, double* rms) try {
    if (!c) return fail(nullptr, PCPF_EINVAL, "precond_info: NULL context");
    if (c->pc_iters < 0) return fail(nullptr, PCPF_ESTATE, "no preconditioning has run");
    if (iters) *iters = c->pc_iters;
    if (rms) *rms = c->pc_rms;
    return PCPF_OK;
} catch (...) {
    return out_of_memory(nullptr);
}

pcpf_status pcpf_residual(pcpf_ctx* c, const void* d_phi, const void* d_psi, double t,
                          int32_t mode, void* d_rphi, void* d_rpsi) try {
    if (check_ctx(c) != PCPF_OK) return PCPF_EINVAL;
    if (mode != PCPF_MODE_PHYS && mode != PCPF_MODE_PRECOND)
        return fail(&c->err, PCPF_EINVAL, "unknown residual mode");
    if (!d_psi || !d_rpsi || (mode == PCPF_MODE_PHYS && (!d_phi || !d_rphi)))
        return fail(&c->err, PCPF_EINVAL, "residual: NULL input or output");
    if (mode == PCPF_MODE_PRECOND && !c->has_sign)
        return fail(&c->err, PCPF_ESTATE, "precond residual needs the sign of a reset");
    if (d_rpsi == d_psi || d_rpsi == d_phi || (d_rphi && (d_rphi == d_phi || d_rphi == d_psi)))
        return fail(&c->err, PCPF_EINVAL, "residual outputs may not alias inputs");
    return DISPATCH(c, residual_impl, d_phi, d_psi, t, mode, d_rphi, d_rpsi);
} catch (...) {
    return out_of_memory(c);
}

pcpf_status pcpf_get_sign(pcpf_ctx* c, void* d_sgn) try {
    if (check_ctx(c) != PCPF_OK) return PCPF_EINVAL;
    if (!c->has_sign) return fail(&c->err, PCPF_ESTATE, "no reset has run");
    if (!d_sgn) return fail(&c->err, PCPF_EINVAL, "d_sgn is NULL");
    const size_t bytes = (size_t)c->mi.E * c->mi.nu * (c->prm.precision != PCPF_FP64 ? 4 : 8);
    HIPCHK(c, hipMemcpyAsync(d_sgn, c->ws + c->L.sgn, bytes, hipMemcpyDeviceToDevice, c->stream));
    return PCPF_OK;
} catch (...) {
    return out_of_memory(c);
}

pcpf_status pcpf_sensor(pcpf_ctx* c, const void* d_psi, void* d_nu) try {
    if (check_ctx(c) != PCPF_OK) return PCPF_EINVAL;
    if (!d_psi || !d_nu) return fail(&c->err, PCPF_EINVAL, "sensor: NULL pointer");
    return DISPATCH(c, sensor_impl, d_psi, d_nu);
} catch (...) {
    return out_of_memory(c);
}

pcpf_status pcpf_reduce(pcpf_ctx* c, int32_t what, const void* d_field, const void* d_ref,
                        double* out) try {
    if (check_ctx(c) != PCPF_OK) return PCPF_EINVAL;
    if (!out) return fail(&c->err, PCPF_EINVAL, "out is NULL");
    if (what != PCPF_REDUCE_MASS && what != PCPF_REDUCE_L1 && what != PCPF_REDUCE_RMS)
        return fail(&c->err, PCPF_EINVAL, "unknown reduction");
    if (what != PCPF_REDUCE_MASS && !d_ref)
        return fail(&c->err, PCPF_EINVAL, "L1 and RMS need d_ref");
    if (!d_field && !c->has_state) return fail(&c->err, PCPF_ESTATE, "no state set");
    return DISPATCH(c, reduce_impl, what, d_field, d_ref, out);
} catch (...) {
    return out_of_memory(c);
}

pcpf_status pcpf_set_timing(pcpf_ctx* c, int32_t on) try {
    if (check_ctx(c) != PCPF_OK) return PCPF_EINVAL;
    if (c->ev_used) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        pcpf_status st = collect_times(c);
        if (st != PCPF_OK) return st;
    }
    c->timing = on != 0;
    return PCPF_OK;
} catch (...) {
    return out_of_memory(c);
}

pcpf_status pcpf_kernel_times(pcpf_ctx* c, double* ms, int64_t* launches, int32_t reset) try {
    if (check_ctx(c) != PCPF_OK) return PCPF_EINVAL;
    for (int k = 0; k < PCPF_KT_COUNT; ++k) {
        if (ms) ms[k] = c->kt_ms[k];
        if (launches) launches[k] = c->kt_n[k];
        if (reset) {
            c->kt_ms[k] = 0.0;
            c->kt_n[k] = 0;
        }
    }
    return PCPF_OK;
} catch (...) {
    return out_of_memory(c);
}

pcpf_status pcpf_set_velocity_amplitude(pcpf_ctx* c, double amp) try {
    if (check_ctx(c) != PCPF_OK) return PCPF_EINVAL;
    if (!std::isfinite(amp)) return fail(&c->err, PCPF_EINVAL, "amplitude must be finite");
    c->prm.vel_amp = amp;
    return PCPF_OK;
} catch (...) {
    return out_of_memory(c);
}

pcpf_status pcpf_ckpt_bytes(const pcpf_ctx* c, int64_t nsteps, int64_t every, size_t* nbytes) try {
    if (!c || !nbytes) return fail(nullptr, PCPF_EINVAL, "ckpt_bytes: NULL argument");
    if (nsteps < 1 || every < 1) return fail(nullptr, PCPF_EINVAL, "nsteps and every must be >= 1");
    const size_t r = c->prm.precision != PCPF_FP64 ? 4 : 8;
    *nbytes = (size_t)((nsteps + every - 1) / every) * 2 * (size_t)c->mi.E * c->mi.nu * r;
    return PCPF_OK;
} catch (...) {
    return out_of_memory(nullptr);
}

pcpf_status pcpf_forward_ckpt(pcpf_ctx* c, double dt, int64_t nsteps, int64_t every, void* d_ckpt,
                              size_t ckpt_bytes) try {
    if (check_ctx(c) != PCPF_OK) return PCPF_EINVAL;
    if (c->mi.shape != PCPF_SHAPE_TENSOR)
        return fail(&c->err, PCPF_EUNSUPPORTED, "the adjoint is built for quadrilaterals and hexahedra");
    if (c->prm.precision == PCPF_BF16)
        return fail(&c->err, PCPF_EUNSUPPORTED, "no adjoint of the PCPF_BF16 form");
    if (c->prm.normal_mode == PCPF_NORMAL_PHI)
        return fail(&c->err, PCPF_EUNSUPPORTED, "no adjoint of the PCPF_NORMAL_PHI form");
    if (c->prm.sgn_mode != PCPF_SGN_PSI0 || c->prm.stop_mode != PCPF_STOP_FIXED)
        return fail(&c->err, PCPF_EUNSUPPORTED,
                    "the adjoint differentiates the PCPF_SGN_PSI0 sign with PCPF_STOP_FIXED");
    if (!c->has_state) return fail(&c->err, PCPF_ESTATE, "no state set");
    size_t need = 0;
    if (pcpf_ckpt_bytes(c, nsteps, every, &need) != PCPF_OK || !std::isfinite(dt))
        return fail(&c->err, PCPF_EINVAL, "bad dt, nsteps or every");
    if (!d_ckpt || ckpt_bytes < need) return fail(&c->err, PCPF_EINVAL, "checkpoint buffer too small");
    const int N = c->prm.reset_every;
    if (N > 0 && every > N)
        return fail(&c->err, PCPF_EINVAL, "checkpoint interval must not exceed reset_every");
    if (N > 0 && !c->has_psi && c->step % N != 0 && nsteps > 1)
        return fail(&c->err, PCPF_EINVAL, "a forced reset off the reset schedule is not supported");
    return DISPATCH(c, forward_ckpt_impl, dt, nsteps, every, d_ckpt);
} catch (...) {
    return out_of_memory(c);
}

pcpf_status pcpf_adjoint_bytes(const pcpf_ctx* c, int64_t every, size_t* nbytes) try {
    if (!c || !nbytes) return fail(nullptr, PCPF_EINVAL, "adjoint_bytes: NULL argument");
    if (every < 1) return fail(nullptr, PCPF_EINVAL, "every must be >= 1");
    if (c->mi.shape != PCPF_SHAPE_TENSOR)
        return fail(nullptr, PCPF_EUNSUPPORTED, "the adjoint is built for quadrilaterals and hexahedra");
    *nbytes = adj_layout(c, every).total;
    return PCPF_OK;
} catch (...) {
    return out_of_memory(nullptr);
}

pcpf_status pcpf_adjoint(pcpf_ctx* c, const void* d_ckpt, void* d_scratch, size_t scratch_bytes,
                         const void* d_gphi, const void* d_gpsi, void* d_gphi0, void* d_gpsi0,
                         double* g_amp) try {
    if (check_ctx(c) != PCPF_OK) return PCPF_EINVAL;
    if (!c->ck_valid) return fail(&c->err, PCPF_ESTATE, "no checkpointed forward run");
    if (!d_ckpt || !d_gphi || !d_gphi0) return fail(&c->err, PCPF_EINVAL, "adjoint: NULL argument");
    if (!d_scratch || scratch_bytes < adj_layout(c, c->ck_every).total)
        return fail(&c->err, PCPF_EINVAL, "adjoint scratch smaller than pcpf_adjoint_bytes");
    if (reinterpret_cast<uintptr_t>(d_scratch) % 256 != 0)
        return fail(&c->err, PCPF_EINVAL, "adjoint scratch must be 256-byte aligned");
    return DISPATCH(c, adjoint_impl, d_ckpt, d_scratch, d_gphi, d_gpsi, d_gphi0, d_gpsi0, g_amp);
} catch (...) {
    return out_of_memory(c);
}

pcpf_status pcpf_adjoint_static(pcpf_ctx* c, const void* d_ckpt, const void* d_gphi,
                                const void* d_gpsi, void* d_gphi0, void* d_gpsi0,
                                double* g_amp) try {
    if (check_ctx(c) != PCPF_OK) return PCPF_EINVAL;
    if (!c->ck_valid) return fail(&c->err, PCPF_ESTATE, "no checkpointed forward run");
    if (!d_ckpt || !d_gphi || !d_gphi0) return fail(&c->err, PCPF_EINVAL, "adjoint: NULL argument");
    const size_t need = adj_layout(c, c->ck_every).total;
    if (need > (size_t)PCPF_ADJOINT_STATIC_BYTES)
        return fail(&c->err, PCPF_EINVAL,
                    "pcpf_adjoint_static: this run needs " + std::to_string(need) +
                        " bytes of adjoint scratch, above the static " +
                        std::to_string((size_t)PCPF_ADJOINT_STATIC_BYTES) +
                        " (checkpoint more often, or pass caller memory to pcpf_adjoint)");
    void* ptr = nullptr;
    pcpf_status st = static_scratch(c, &ptr);
    if (st != PCPF_OK) return st;
    // per-launch timing creates HIP events: off for the duration of the call
    struct NoTiming {
        pcpf_ctx* c;
        bool was;
        ~NoTiming() { c->timing = was; }
    } keep{c, c->timing};
    c->timing = false;
    return DISPATCH(c, adjoint_impl, d_ckpt, ptr, d_gphi, d_gpsi, d_gphi0, d_gpsi0, g_amp);
} catch (...) {
    return out_of_memory(c);
}

}  // extern "C"
