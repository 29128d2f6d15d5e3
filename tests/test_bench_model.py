"""The byte model behind bench.py's roofline figures, checked on the CPU.

B_alg per DOF-stage (5 V N_u RK4 register values + 2 V N_f face-exchange values per element,
over N_u) against the per-configuration values 14.0 / 13.2 / 16.0 / 14.8 of the 2D p=3,
2D p=4, 3D p=3 and 3D p=4 workloads, and the words the two launches of a stage move
against a count written out from their argument lists (each array read or written once
per launch)."""
import math
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("d,p,values", [(2, 3, 14.0), (2, 4, 13.2), (3, 3, 16.0), (3, 4, 14.8)])
def test_stage_alg_words_per_dof(d, p, values):
    nu = (p + 1) ** d
    assert math.isclose(bench.stage_words(d, p)["alg"] / nu, values, rel_tol=1e-12)


@pytest.mark.parametrize("d,p", [(2, 3), (2, 4), (3, 3), (3, 4)])
@pytest.mark.parametrize("lifted", [False, True])
@pytest.mark.parametrize("tables", [False, True])
def test_stage_impl_words(d, p, lifted, tables):
    n = p + 1
    nu, nfa = n ** d, n ** (d - 1)
    geo = d + 2 * d * d + 1          # x0, J, J^-1, |J|
    adj = 2 * d / 2                  # 2 d int32 neighbour indices per element, in words
    tab = 2 * d * (n + 2) if tables else 0   # (sin^2, sin 2x) at n nodes + 2 ends per axis
    # grad_flux: reads u (2 planes), the + face traces (2 d planes of nfa), geo, the
    # adjacency and the velocity tables; writes P (2 planes) and the + face common fluxes
    # (one slot per + face point, 2 d planes of nfa)
    gf = 2 * nu + 2 * d * nfa + geo + adj + tab + 2 * nu + 2 * d * nfa
    # update, averaged over the 4 stages: reads P, the - face fluxes (and the + face ones
    # unless the line kernel lifted them into P), |J|, the adjacency, u_n and acc (not on
    # stage 1); writes acc (not on stage 4), the next stage input and the pushed traces
    up = 2 * nu + (1 if lifted else 2) * 2 * d * nfa + 1 + adj + 2 * nu + 0.75 * 2 * nu \
        + 0.75 * 2 * nu + 2 * nu + 2 * d * nfa
    w = bench.stage_words(d, p, lifted=lifted, tables=tables)
    assert w["grad_flux"] == gf and w["update"] == up and w["impl"] == gf + up
    # 96^3 p=4 FP64: 13.1 GB of algorithmic bytes per stage
    if (d, p) == (3, 4):
        assert abs(w["alg"] * 8 * 96 ** 3 / 1e9 - 13.095) < 1e-3


def test_stage_words_of_forms():
    """Which kernels run: the line kernel (3D in FP64 and FP32, 2D in FP32, and in FP64 from
    p = 4) lifts the + face fluxes; the BF16 form and 2D FP64 below p = 4 do not; the box
    workloads with trigonometric fields read the velocity tables, the uniform-velocity one
    does not."""
    import workloads as W
    c5, c2, c1 = W.config("C5"), W.config("C2"), W.config("C1")
    assert bench.stage_words_of(c5, "fp64") == bench.stage_words(3, 4, lifted=True, tables=True)
    assert bench.stage_words_of(c5, "bf16") == bench.stage_words(3, 4, lifted=False, tables=True)
    assert bench.stage_words_of(c2, "fp64") == bench.stage_words(2, 4, lifted=True, tables=True)
    assert bench.stage_words_of(c2, "fp32") == bench.stage_words(2, 4, lifted=True, tables=True)
    assert bench.stage_words_of(c1, "fp64") == bench.stage_words(2, 3, lifted=False, tables=False)


@pytest.mark.parametrize("p", [3, 4, 5])
def test_triangle_stage_words(p):
    """Triangles: N_u = (p+1)(p+2)/2 and N_f = 3(p+1) in the same B_alg formula; the
    launches' words counted from their arrays (each flux point has its own trace and flux
    slot, the slot table is one 4-byte code per point)."""
    nu, nf = (p + 1) * (p + 2) // 2, 3 * (p + 1)
    w = bench.stage_words(2, p, "triangle")
    assert w["alg"] == 10 * nu + 4 * nf
    # grad_flux: u, own + partner traces, geometry (11), codes; writes P and the owned half
    # of the common fluxes
    gf = 2 * nu + 2 * 2 * nf + 11 + nf / 2 + 2 * nu + nf
    # update: P, the flux of every point, geometry, codes, u_n, acc (3 of 4 stages);
    # writes acc (3 of 4), the next stage input, the own traces
    up = 2 * nu + 2 * nf + 11 + nf / 2 + 2 * nu + 1.5 * nu + 1.5 * nu + 2 * nu + 2 * nf
    assert w["grad_flux"] == gf and w["update"] == up
    if p == 4:
        # 1024^2 cells, 2 097 152 triangles: FP64 B_alg per stage
        assert abs(w["alg"] * 8 * 2 * 1024 ** 2 / 1e9 - (210 * 8 * 2 * 1024 ** 2) / 1e9) < 1e-9


def test_triangle_mfma_flops():
    """The matrix-core flops of one launch of the triangle MFMA grad_flux: 18 operator
    products per 16-element tile (Steps 1-3: M0 u and, per direction, D_k u and the lifted
    jump, for both variables; Step 5: M0 of the two gradient components of both variables;
    Step 6: DH_0 and DH_1 for both variables), each four 16 x 16 x 4 instructions of 2048
    flops; none for tensor elements or orders above 4."""
    import workloads as W
    t2 = W.config("T2")
    tiles = (t2.nelem + 15) // 16
    assert bench.TRI_MFMA_PER_TILE == (2 * (1 + 2 * 2) + 2 * 2 + 2 * 2) * 4
    assert bench.tri_mfma_flops(t2, "fp64") == tiles * 72 * 2048
    assert bench.tri_mfma_flops(t2, "bf16") is None
    assert bench.tri_mfma_flops(W.config("C5"), "fp64") is None
