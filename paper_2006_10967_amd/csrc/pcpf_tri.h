// Triangle element of the FR-PCPF library: block shape of its kernels and the layout of its
// dense operator block.
#pragma once

#include "pcpf_internal.h"

namespace pcpf {

// Order-p triangle: N_u = (p+1)(p+2)/2 solution points, N_f = 3(p+1) flux points; a block
// of 256 threads holds EPB = floor(256 / max(N_u, N_f)) elements.
template <int P>
struct TriShape {
    static constexpr int NU = (P + 1) * (P + 2) / 2;
    static constexpr int NF = 3 * (P + 1);
    static constexpr int NM = NU > NF ? NU : NF;
    static constexpr int EPB = 256 / NM;
    static constexpr int G = 11;             // x0[2], J[2][2], Jinv[2][2], det J
    // operator block (compute type), row-major:
    static constexpr int OM0 = 0;                    // M0[N_f][N_u]      interpolation
    static constexpr int OD0 = OM0 + NF * NU;        // D_0[N_u][N_u]     d/dxi_0
    static constexpr int OD1 = OD0 + NU * NU;        // D_1[N_u][N_u]     d/dxi_1
    static constexpr int OL = OD1 + NU * NU;         // Lift[N_u][N_f]    correction divergence
    static constexpr int OVI = OL + NU * NF;         // Vinv[N_u][N_u]    nodal -> modal
    static constexpr int OTOP = OVI + NU * NU;       // topmask[N_u]      1 on degree-p modes
    static constexpr int OUR = OTOP + NU;            // solution points [N_u][2]
    static constexpr int OFR = OUR + 2 * NU;         // flux points [N_f][2]
    static constexpr int ONH = OFR + 2 * NF;         // reference outward unit normals [N_f][2]
    static constexpr int ODH0 = ONH + 2 * NF;        // DH_k = D_k - Lift diag(nhat_k) M0,
    static constexpr int ODH1 = ODH0 + NU * NU;      //   [N_u][N_u] each (Step 6 volume part)
    static constexpr int NOPS = ODH1 + NU * NU;
};

constexpr int tri_nupts(int p) { return (p + 1) * (p + 2) / 2; }
constexpr int tri_nfpts(int p) { return 3 * (p + 1); }
constexpr int tri_ops_size(int p) {
    return tri_nfpts(p) * tri_nupts(p) * 2 + 5 * tri_nupts(p) * tri_nupts(p) + tri_nupts(p) +
           2 * tri_nupts(p) + 4 * tri_nfpts(p);
}
constexpr int TRI_MAX_ORDER = 5;

template <typename R>
bool get_tri_launchers(int p, Launchers<R>* out);

}  // namespace pcpf
