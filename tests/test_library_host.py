"""Host-side checks of the HIP library (no GPU needed): the library loads and exports every
function of include/pcpf.h, its host builders agree with the oracle's independent
construction, and invalid meshes / parameters are rejected before any device work."""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import Oracle
from oracle.basis import Basis1D

P = pytest.importorskip("paper_2006_10967_amd")
from paper_2006_10967_amd import _lib  # noqa: E402
from paper_2006_10967_amd.solver import MeshArgs, make_params  # noqa: E402


def test_exports_every_declared_symbol():
    lib = _lib.load()
    names = _lib.header_functions()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert lib.pcpf_abi_version() == _lib.ABI_VERSION == 2


def test_missing_library_fails_loudly(tmp_path):
    """There is no fallback: without the built library the binding raises instead of
    computing anything (checked in a fresh process, since the path is read at import)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, PCPF_LIBRARY=str(tmp_path / "absent" / "libpcpf.so"))
    code = ("from paper_2006_10967_amd import _lib\n"
            "try:\n    _lib.load()\nexcept ImportError as e:\n    print('raised:', e)\n")
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=root, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert "raised:" in r.stdout and "missing" in r.stdout, r.stdout


def test_binding_constants_match_the_header():
    """Every PCPF_* constant that the binding defines has the header's value."""
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "include", "pcpf.h")).read()
    values = {m.group(1): int(m.group(2))
              for m in re.finditer(r"\b(PCPF_[A-Z0-9_]+)\s*=\s*(\d+)", hdr)}
    assert "PCPF_ENOMEM" in values
    checked = 0
    for name in dir(_lib):
        if name.startswith("PCPF_") and name in values:
            assert getattr(_lib, name) == values[name], name
            checked += 1
    assert checked >= 20
    assert set(_lib.STATUS_NAMES) == {v for k, v in values.items()
                                      if k == "PCPF_OK" or re.fullmatch(r"PCPF_E[A-Z]+", k)}


@pytest.mark.parametrize("p", range(1, 7))
def test_line_operators_match_oracle_basis(p):
    ops = P.line_operators(p)
    b = Basis1D(p)
    n = p + 1
    assert np.max(np.abs(ops["nodes"] - b.xi)) < 1e-15
    assert np.max(np.abs(ops["weights"] - b.w)) < 1e-14
    D = ops["deriv"].reshape(n, n)
    assert np.max(np.abs(D - b.dlagrange(b.xi))) < 1e-12
    assert np.max(np.abs(ops["lminus"] - b.lagrange(-1.0)[0])) < 1e-13
    assert np.max(np.abs(ops["lplus"] - b.lagrange(1.0)[0])) < 1e-13
    # correction-function derivatives: the oracle's Radau polynomials (FR definition)
    assert np.max(np.abs(ops["cplus"] - b.dg_right(b.xi))) < 1e-11
    assert np.max(np.abs(ops["cminus"] + b.dg_left(b.xi))) < 1e-11
    # modal transform inverts the oracle's Vandermonde (modes x points)
    Vi = ops["vinv"].reshape(n, n)
    assert np.max(np.abs(Vi @ b.V.T - np.eye(n))) < 1e-13


@pytest.mark.parametrize("d,p,shape,kw", [
    (2, 3, (5, 4), {}),
    (2, 4, (4, 4), {"shear": 0.25}),
    (3, 2, (3, 4, 2), {"perturb": 0.2}),
    (3, 3, (2, 2, 3), {"periodic": False}),
])
def test_solution_coords_and_adjacency_match_oracle(d, p, shape, kw):
    mesh, prm = W.small_case(d, p, shape, **kw)
    o = Oracle(d, p, mesh, prm)
    m = MeshArgs(d, p, mesh.x0, mesh.jac, mesh.nbr, _period(mesh))
    xs = m.solution_coords()
    assert np.max(np.abs(xs - o.disc.xs)) < 1e-14
    # the adjacency table agrees with the oracle's pairing of flux points by coordinates
    ops = o.ops
    nfa = ops.nfpts_face
    for e in range(mesh.nelem):
        for f in range(2 * d):
            j0 = f * nfa
            en = mesh.nbr[e, f]
            has = o.disc.has_pair[e, j0:j0 + nfa]
            if en < 0:
                assert not has.any()
            else:
                assert has.all()
                assert np.all(o.disc.pair_e[e, j0:j0 + nfa] == en)
                fo = f ^ 1
                assert np.all(o.disc.pair_j[e, j0:j0 + nfa] == fo * nfa + np.arange(nfa))


def _period(mesh):
    return [float(mesh.period[k]) if mesh.periodic[k] else 0.0 for k in range(mesh.ndims)]


def _create_status(mesh_args, params, ws=1, nbytes=1 << 30):
    lib = _lib.load()
    ctx = ctypes.c_void_p()
    st = lib.pcpf_create(ctypes.byref(mesh_args.c), ctypes.byref(params), ctypes.c_void_p(ws * 256),
                         ctypes.c_size_t(nbytes), None, ctypes.byref(ctx))
    return st, lib.pcpf_last_error(None).decode()


def test_create_rejects_invalid_input_before_device_work():
    mesh, prm = W.small_case(2, 3, (4, 4))
    good = make_params(prm, "fp64")
    # non-reciprocal adjacency
    nbr = mesh.nbr.copy()
    nbr[0, 1] = 2
    st, msg = _create_status(MeshArgs(2, 3, mesh.x0, mesh.jac, nbr, _period(mesh)), good)
    assert st == _lib.PCPF_EINVAL and "reciprocal" in msg
    # mismatched face points
    x0 = mesh.x0.copy()
    x0[5, 1] += 0.01
    st, msg = _create_status(MeshArgs(2, 3, x0, mesh.jac, mesh.nbr, _period(mesh)), good)
    assert st == _lib.PCPF_EINVAL and "coincide" in msg
    # inverted element
    jac = mesh.jac.copy()
    jac[3] *= -1
    st, msg = _create_status(MeshArgs(2, 3, mesh.x0, jac, mesh.nbr, _period(mesh)), good)
    assert st == _lib.PCPF_EINVAL
    # bad parameters
    bad = make_params(prm, "fp64")
    bad.kappa = 0.0
    st, _ = _create_status(MeshArgs(2, 3, mesh.x0, mesh.jac, mesh.nbr, _period(mesh)), bad)
    assert st == _lib.PCPF_EINVAL
    bad = make_params(prm, "fp64")
    bad.precision = 7
    st, _ = _create_status(MeshArgs(2, 3, mesh.x0, mesh.jac, mesh.nbr, _period(mesh)), bad)
    assert st == _lib.PCPF_EUNSUPPORTED
    # unknown sign and stop modes
    for field in ("sgn_mode", "stop_mode", "normal_mode"):
        bad = make_params(prm, "fp64")
        setattr(bad, field, 2)
        st, msg = _create_status(MeshArgs(2, 3, mesh.x0, mesh.jac, mesh.nbr, _period(mesh)), bad)
        assert st == _lib.PCPF_EINVAL and field in msg, (field, msg)
    # an empty mesh
    m0 = MeshArgs(2, 3, mesh.x0, mesh.jac, mesh.nbr, _period(mesh))
    m0.c.nelem = 0
    st, msg = _create_status(m0, good)
    assert st == _lib.PCPF_EINVAL and "nelem" in msg
    # workspace too small / misaligned
    st, _ = _create_status(MeshArgs(2, 3, mesh.x0, mesh.jac, mesh.nbr, _period(mesh)), good, nbytes=16)
    assert st == _lib.PCPF_EINVAL
    lib = _lib.load()
    ctx = ctypes.c_void_p()
    st = lib.pcpf_create(ctypes.byref(MeshArgs(2, 3, mesh.x0, mesh.jac, mesh.nbr, _period(mesh)).c),
                         ctypes.byref(good), ctypes.c_void_p(257), ctypes.c_size_t(1 << 30), None,
                         ctypes.byref(ctx))
    assert st == _lib.PCPF_EINVAL
    # order out of range
    ops = P.line_operators(3)
    with pytest.raises(P.PcpfError):
        P.line_operators(7)
    m = MeshArgs(3, 3, np.zeros((1, 3)), np.eye(3)[None], -np.ones((1, 6)),
                 ops=P.line_operators(3))
    m.c.order = 6
    st, _ = _create_status(m, good)
    assert st == _lib.PCPF_EUNSUPPORTED


def test_workspace_bytes_scale_with_precision():
    lib = _lib.load()
    mesh, prm = W.small_case(3, 3, (4, 4, 4))
    m = MeshArgs(3, 3, mesh.x0, mesh.jac, mesh.nbr, _period(mesh))
    sizes = []
    for prec in ("fp64", "fp32"):
        nb = ctypes.c_size_t()
        assert lib.pcpf_workspace_bytes(ctypes.byref(m.c), ctypes.byref(make_params(prm, prec)),
                                        ctypes.byref(nb)) == 0
        sizes.append(nb.value)
    assert sizes[1] < sizes[0] < 2.2 * sizes[1]
    # five state registers + three face fields dominate
    E, nu, nfa = 64, 64, 16
    assert sizes[0] >= 8 * (5 * 2 * E * nu + 3 * 2 * E * 3 * nfa)


def test_meshes_beyond_32_bit_array_offsets_are_refused():
    """Every per-element array must stay below 4 GiB (the kernels use 32-bit byte
    offsets): a 3D p=5 mesh of 3 M elements (216 points each) is refused before any
    array is read, and the 96^3 p=4 workload is accepted."""
    lib = _lib.load()
    prm = make_params(W.small_case(3, 5, (1, 1, 1))[1], "fp64")
    m = MeshArgs(3, 5, np.zeros((1, 3)), np.eye(3)[None], -np.ones((1, 6)),
                 ops=P.line_operators(5))
    m.c.nelem = 3_000_000
    nb = ctypes.c_size_t()
    st = lib.pcpf_workspace_bytes(ctypes.byref(m.c), ctypes.byref(prm), ctypes.byref(nb))
    assert st == _lib.PCPF_EUNSUPPORTED
    assert "4 GiB" in lib.pcpf_last_error(None).decode()
    m.c.order = 4
    m.c.nelem = 96 ** 3
    m4 = MeshArgs(3, 4, np.zeros((1, 3)), np.eye(3)[None], -np.ones((1, 6)),
                  ops=P.line_operators(4))
    m4.c.nelem = 96 ** 3
    st = lib.pcpf_workspace_bytes(ctypes.byref(m4.c), ctypes.byref(prm), ctypes.byref(nb))
    assert st == _lib.PCPF_OK and nb.value > 10 * 2 ** 30
