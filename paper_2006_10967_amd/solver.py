"""Python binding of the FR-PCPF HIP library (argument marshalling only).

Every step of the method runs in the library's kernels; this module converts numpy /
torch arguments to the C ABI of include/pcpf.h. torch provides the device memory (the
workspace and the state tensors) and the HIP stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import PcpfDenseMesh, PcpfMesh, PcpfParams, check

FP64, FP32, BF16 = _lib.PCPF_FP64, _lib.PCPF_FP32, _lib.PCPF_BF16
MODE_PHYS, MODE_PRECOND = _lib.PCPF_MODE_PHYS, _lib.PCPF_MODE_PRECOND
REDUCE_MASS, REDUCE_L1, REDUCE_RMS = _lib.PCPF_REDUCE_MASS, _lib.PCPF_REDUCE_L1, _lib.PCPF_REDUCE_RMS

_PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16, FP64: FP64, FP32: FP32, BF16: BF16}
_DTYPES = {FP64: torch.float64, FP32: torch.float32, BF16: torch.float32}


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def line_operators(order: int) -> dict:
    """1D Gauss-Legendre element operators built by the library (host)."""
    lib = _lib.load()
    n = order + 1
    out = {k: np.zeros(n) for k in ("nodes", "weights", "lminus", "lplus", "cminus", "cplus")}
    out["deriv"] = np.zeros(n * n)
    out["vinv"] = np.zeros(n * n)
    check(lib.pcpf_line_operators(order, _dptr(out["nodes"]), _dptr(out["weights"]),
                                  _dptr(out["deriv"]), _dptr(out["lminus"]), _dptr(out["lplus"]),
                                  _dptr(out["cminus"]), _dptr(out["cplus"]), _dptr(out["vinv"])))
    return out


def triangle_operators(order: int) -> dict:
    """Dense operators of the library's order-p triangle element (host)."""
    lib = _lib.load()
    nu, nf = (order + 1) * (order + 2) // 2, 3 * (order + 1)
    out = {"upt_ref": np.zeros((nu, 2)), "fpt_ref": np.zeros((nf, 2)), "M0": np.zeros((nf, nu)),
           "D": np.zeros((2, nu, nu)), "LiftN": np.zeros((2, nu, nf)), "Lift": np.zeros((nu, nf)),
           "Vinv": np.zeros((nu, nu)), "topmask": np.zeros(nu, dtype=np.uint8), "W": np.zeros(nu),
           "ref_fnorm": np.zeros((nf, 2))}
    check(lib.pcpf_triangle_operators(
        order, *[_dptr(out[k]) for k in ("upt_ref", "fpt_ref", "M0", "D", "LiftN", "Lift", "Vinv")],
        out["topmask"].ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _dptr(out["W"]),
        _dptr(out["ref_fnorm"])))
    return out


class MeshArgs:
    """A pcpf_mesh whose host arrays stay alive as long as this object."""

    def __init__(self, ndims: int, order: int, x0, jac, nbr, period=(0.0, 0.0, 0.0),
                 ops: dict | None = None):
        self.ops = ops if ops is not None else line_operators(order)
        self.x0 = np.ascontiguousarray(x0, dtype=np.float64)
        self.jac = np.ascontiguousarray(jac, dtype=np.float64)
        self.nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        E = self.x0.shape[0]
        if self.x0.shape != (E, ndims) or self.jac.shape != (E, ndims, ndims) \
                or self.nbr.shape != (E, 2 * ndims):
            raise ValueError("mesh array shapes do not match ndims")
        o = self.ops
        self.c = PcpfMesh(ndims, order, E, _dptr(o["nodes"]), _dptr(o["weights"]),
                          _dptr(o["deriv"]), _dptr(o["lminus"]), _dptr(o["lplus"]),
                          _dptr(o["cminus"]), _dptr(o["cplus"]), _dptr(o["vinv"]),
                          _dptr(self.x0), _dptr(self.jac),
                          self.nbr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          (ctypes.c_double * 3)(*[float(x) for x in (list(period) + [0.0] * 3)[:3]]))
        self.ndims, self.order, self.nelem = ndims, order, E
        self.nupts = (order + 1) ** ndims

    def solution_coords(self) -> np.ndarray:
        lib = _lib.load()
        xs = np.zeros((self.nelem, self.nupts, self.ndims))
        check(lib.pcpf_solution_coords(ctypes.byref(self.c), _dptr(xs)))
        return xs


# LDG switch vector of the triangle meshes: on an interior edge the owner (beta = +1/2, the
# side that takes the neighbour's trace in the common solution and computes the common flux)
# is the side whose outward normal has a positive component along it. Any fixed vector
# not parallel to an edge of the mesh gives a valid LDG orientation; this one is parallel to
# no edge of a split-Cartesian mesh (axis-aligned and diagonal edges).
TRI_SWITCH = np.array([1.0, 1.0 / np.sqrt(2.0)])


class DenseMeshArgs:
    """A pcpf_dense_mesh (the dense operators, per-element geometry and per-flux-point
    connectivity of the method's statement) whose host arrays stay alive as long as this
    object. Arrays are given as numpy arrays of the shapes in include/pcpf.h; ``jac`` is
    optional."""

    _F64 = ("M0", "D", "LiftN", "Lift", "Vinv", "W", "ref_fnorm", "jinv", "detj", "fnorm",
            "fscale", "xorig")

    def __init__(self, ndims, order, nelem, nupts, nfpts, arrays: dict, period=(0.0, 0.0, 0.0),
                 shape=_lib.PCPF_SHAPE_TENSOR):
        self.keep = {}
        c = PcpfDenseMesh()
        c.ndims, c.order, c.shape = int(ndims), int(order), int(shape)
        c.nupts, c.nfpts, c.nelem = int(nupts), int(nfpts), int(nelem)
        for name in self._F64:
            a = np.ascontiguousarray(arrays[name], dtype=np.float64)
            self.keep[name] = a
            setattr(c, name, _dptr(a))
        jac = arrays.get("jac")
        if jac is not None:
            a = np.ascontiguousarray(jac, dtype=np.float64)
            self.keep["jac"] = a
            c.jac = _dptr(a)
        for name in ("topmask", "owner"):
            a = np.ascontiguousarray(arrays[name], dtype=np.uint8)
            self.keep[name] = a
            setattr(c, name, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        a = np.ascontiguousarray(arrays["nbr_slot"], dtype=np.int32)
        self.keep["nbr_slot"] = a
        c.nbr_slot = a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        c.period = (ctypes.c_double * 3)(*[float(x) for x in (list(period) + [0.0] * 3)[:3]])
        self.c = c
        self.ndims, self.order, self.nelem, self.nupts = int(ndims), int(order), int(nelem), int(nupts)

    @classmethod
    def from_triangles(cls, mesh, order: int, ops: dict | None = None) -> "DenseMeshArgs":
        """The dense description of a triangle mesh (x0 [E, 2], jac [E, 2, 2] of the maps
        x = x0 + J (r, s), the flux-point pairing of ``mesh.slot_pairs(order + 1)``, periods):
        the library's triangle operators (or given ones), J^-1, det J, unit normals
        J^-T nhat / |J^-T nhat| and face scales det J |J^-T nhat| per flux point, owners by
        TRI_SWITCH (boundary points owned)."""
        ops = ops or triangle_operators(order)
        nu, nf = ops["W"].size, ops["M0"].shape[0]
        jac = np.asarray(mesh.jac, dtype=np.float64)
        jinv = np.linalg.inv(jac)
        det = np.linalg.det(jac)
        nr = np.einsum("eki,fk->efi", jinv, ops["ref_fnorm"])
        mag = np.linalg.norm(nr, axis=-1)
        fnorm = nr / mag[..., None]
        nbr_slot = np.asarray(mesh.slot_pairs(order + 1))
        owner = np.where(nbr_slot >= 0, (fnorm.reshape(-1, 2) @ TRI_SWITCH) > 0, True)
        arr = dict(ops, jinv=jinv, detj=det, fnorm=fnorm, fscale=det[:, None] * mag,
                   xorig=np.asarray(mesh.x0, dtype=np.float64), jac=jac, nbr_slot=nbr_slot,
                   owner=owner)
        period = [float(mesh.period[k]) if mesh.periodic[k] else 0.0 for k in range(2)]
        return cls(2, order, jac.shape[0], nu, nf, arr, period, shape=_lib.PCPF_SHAPE_TRIANGLE)

    def solution_coords(self) -> np.ndarray:
        """Physical coordinates [E, N_u, d] of the solution points of a triangle description
        (x = xorig + J (r, s) at the reference points of pcpf_triangle_operators)."""
        if self.c.shape != _lib.PCPF_SHAPE_TRIANGLE or "jac" not in self.keep:
            raise ValueError("coordinates are given for triangle descriptions with jac")
        upt = triangle_operators(self.order)["upt_ref"]
        return self.keep["xorig"][:, None, :] + np.einsum("eik,uk->eui", self.keep["jac"], upt)

    def workspace_bytes(self, params, precision="fp64") -> int:
        lib = _lib.load()
        nb = ctypes.c_size_t(0)
        cp = make_params(params, _PRECISIONS[precision])
        check(lib.pcpf_workspace_bytes_dense(ctypes.byref(self.c), ctypes.byref(cp), ctypes.byref(nb)))
        return nb.value


def make_params(prm, precision) -> PcpfParams:
    """pcpf_params from any object with the workloads.Params attribute names."""
    c = PcpfParams()
    for name in ("gamma", "eps", "eps_w", "tau", "nu_max", "s0", "kappa", "dtau", "delta_n",
                 "delta_g", "delta_phi", "vel_amp", "vel_period"):
        setattr(c, name, float(getattr(prm, name)))
    u0 = list(getattr(prm, "vel_u0")) + [0.0] * 3
    c.vel_u0 = (ctypes.c_double * 3)(*[float(x) for x in u0[:3]])
    c.vel_kind = int(prm.vel_kind)
    c.reset_mode = int(prm.reset_mode)
    c.reset_every = int(prm.reset_every)
    c.precond_iters = int(prm.precond_iters)
    c.precision = _PRECISIONS[precision]
    c.normal_mode = int(getattr(prm, "normal_mode", 0))
    c.sgn_mode = int(getattr(prm, "sgn_mode", 0))
    c.stop_mode = int(getattr(prm, "stop_mode", 0))
    return c


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Solver:
    """One FR-PCPF context on a CUDA/HIP device."""

    def __init__(self, ndims, order, x0, jac, nbr, params, precision="fp64", device="cuda",
                 period=(0.0, 0.0, 0.0), dense: "DenseMeshArgs | None" = None):
        self.lib = _lib.load()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.dense = dense
        self.mesh = MeshArgs(ndims, order, x0, jac, nbr, period) if dense is None else None
        self.params = params
        self.precision = _PRECISIONS[precision]
        self.dtype = _DTYPES[self.precision]
        self.cparams = make_params(params, self.precision)
        nb = ctypes.c_size_t(0)
        if dense is None:
            check(self.lib.pcpf_workspace_bytes(ctypes.byref(self.mesh.c),
                                                ctypes.byref(self.cparams), ctypes.byref(nb)))
        else:
            check(self.lib.pcpf_workspace_bytes_dense(ctypes.byref(dense.c),
                                                      ctypes.byref(self.cparams), ctypes.byref(nb)))
        self.ws_bytes = nb.value
        with torch.cuda.device(self.device):
            self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            base = self.ws.data_ptr()
            self._ws_ptr = (base + 255) // 256 * 256
            self.stream = torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        if dense is None:
            check(self.lib.pcpf_create(ctypes.byref(self.mesh.c), ctypes.byref(self.cparams),
                                       ctypes.c_void_p(self._ws_ptr), ctypes.c_size_t(self.ws_bytes),
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
            self.nelem = self.mesh.nelem
            self.nupts = self.mesh.nupts
        else:
            check(self.lib.pcpf_create_dense(ctypes.byref(dense.c), ctypes.byref(self.cparams),
                                             ctypes.c_void_p(self._ws_ptr),
                                             ctypes.c_size_t(self.ws_bytes),
                                             ctypes.c_void_p(self.stream.cuda_stream),
                                             ctypes.byref(ctx)))
            self.nelem = dense.nelem
            self.nupts = dense.nupts
        self.ctx = ctx

    @classmethod
    def from_dense(cls, dense: "DenseMeshArgs", params, precision="fp64", device="cuda"):
        """A context from the dense description of pcpf_dense_mesh."""
        return cls(dense.ndims, dense.order, None, None, None, params, precision, device,
                   dense=dense)

    @classmethod
    def from_box(cls, mesh, order, params, precision="fp64", device="cuda"):
        period = [float(mesh.period[k]) if mesh.periodic[k] else 0.0 for k in range(mesh.ndims)]
        return cls(mesh.ndims, order, mesh.x0, mesh.jac, mesh.nbr, params, precision, device,
                   period)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            self.lib.pcpf_destroy(ctx)
            self.ctx = None

    # -- helpers -----------------------------------------------------------------------
    def _field(self, a) -> torch.Tensor:
        t = torch.as_tensor(a)
        if t.shape != (self.nelem, self.nupts):
            raise ValueError(f"field must have shape {(self.nelem, self.nupts)}")
        return t.to(device=self.device, dtype=self.dtype).contiguous()

    def empty(self, shape=None):
        shape = shape or (self.nelem, self.nupts)
        return torch.empty(shape, dtype=self.dtype, device=self.device)

    def _chk(self, status):
        check(status, self.ctx)

    # -- the C ABI ------------------------------------------------------------------------
    def solution_coords(self) -> np.ndarray:
        if self.mesh is None:
            return self.dense.solution_coords()
        return self.mesh.solution_coords()

    @classmethod
    def from_triangles(cls, mesh, order, params, precision="fp64", device="cuda"):
        """A context on a triangle mesh (see DenseMeshArgs.from_triangles)."""
        return cls.from_dense(DenseMeshArgs.from_triangles(mesh, order), params, precision,
                              device)

    def set_state(self, phi, psi=None, t=0.0, step=0):
        self._phi_in = self._field(phi)
        self._psi_in = self._field(psi) if psi is not None else None
        self._chk(self.lib.pcpf_set_state(self.ctx, _ptr(self._phi_in), _ptr(self._psi_in),
                                          float(t), int(step)))

    def get_state(self, want_psi=True):
        phi = self.empty()
        psi = self.empty() if want_psi else None
        t = ctypes.c_double()
        n = ctypes.c_int64()
        self._chk(self.lib.pcpf_get_state(self.ctx, _ptr(phi), _ptr(psi), ctypes.byref(t),
                                          ctypes.byref(n)))
        return phi, psi, t.value, n.value

    def step(self, dt, nsteps=1):
        self._chk(self.lib.pcpf_step(self.ctx, float(dt), int(nsteps)))

    def precondition(self, iters=-1):
        self._chk(self.lib.pcpf_precondition(self.ctx, int(iters)))

    def precond_info(self):
        """(iterations, stop-rule RMS) of the last preconditioning."""
        n = ctypes.c_int32()
        r = ctypes.c_double()
        self._chk(self.lib.pcpf_precond_info(self.ctx, ctypes.byref(n), ctypes.byref(r)))
        return n.value, r.value

    def residual(self, phi, psi, t=0.0, mode=MODE_PHYS):
        phi_t = self._field(phi) if phi is not None else None
        psi_t = self._field(psi)
        rpsi = self.empty()
        rphi = self.empty() if mode == MODE_PHYS else None
        self._chk(self.lib.pcpf_residual(self.ctx, _ptr(phi_t), _ptr(psi_t), float(t), int(mode),
                                         _ptr(rphi), _ptr(rpsi)))
        return rphi, rpsi

    def sign(self):
        out = self.empty()
        self._chk(self.lib.pcpf_get_sign(self.ctx, _ptr(out)))
        return out

    def sensor(self, psi):
        psi_t = self._field(psi)
        nu = self.empty((self.nelem,))
        self._chk(self.lib.pcpf_sensor(self.ctx, _ptr(psi_t), _ptr(nu)))
        return nu

    def reduce(self, what=REDUCE_MASS, field=None, ref=None) -> float:
        f = self._field(field) if field is not None else None
        r = self._field(ref) if ref is not None else None
        out = ctypes.c_double()
        self._chk(self.lib.pcpf_reduce(self.ctx, int(what), _ptr(f), _ptr(r), ctypes.byref(out)))
        return out.value

    def set_timing(self, on=True):
        self._chk(self.lib.pcpf_set_timing(self.ctx, 1 if on else 0))

    def kernel_times(self, reset=False):
        """{class: (total ms, launches)} of the per-launch event timing."""
        ms = (ctypes.c_double * 4)()
        n = (ctypes.c_int64 * 4)()
        self._chk(self.lib.pcpf_kernel_times(self.ctx, ms, n, 1 if reset else 0))
        names = ("grad_flux", "update", "pc_grad_flux", "pc_update")
        return {k: (ms[i], n[i]) for i, k in enumerate(names)}

    def mass(self, field=None) -> float:
        return self.reduce(REDUCE_MASS, field)

    def l1(self, ref, field=None) -> float:
        return self.reduce(REDUCE_L1, field, ref)

    def rms(self, field, ref) -> float:
        return self.reduce(REDUCE_RMS, field, ref)

    # -- adjoint ------------------------------------------------------------------------
    def set_velocity_amplitude(self, amp: float):
        self._chk(self.lib.pcpf_set_velocity_amplitude(self.ctx, float(amp)))

    def forward_ckpt(self, dt, nsteps, every=None):
        """Advance nsteps steps keeping checkpoints every `every` steps (default: the
        reset interval, or the whole run); returns the checkpoint buffer that
        :meth:`adjoint` reads."""
        if every is None:
            every = int(self.cparams.reset_every) or int(nsteps)
            every = min(every, int(nsteps))
        nb = ctypes.c_size_t(0)
        self._chk(self.lib.pcpf_ckpt_bytes(self.ctx, int(nsteps), int(every), ctypes.byref(nb)))
        ck = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        self._run_id = getattr(self, "_run_id", 0) + 1
        self._ckpt, self._ckpt_every = None, None
        self._chk(self.lib.pcpf_forward_ckpt(self.ctx, float(dt), int(nsteps), int(every),
                                             _ptr(ck), ctypes.c_size_t(nb.value)))
        self._ckpt, self._ckpt_every = ck, int(every)
        return ck

    @property
    def run_id(self) -> int:
        """Identifier of the run the context has recorded for :meth:`adjoint` (0: none);
        every :meth:`forward_ckpt` records a new run, replacing the previous one."""
        return getattr(self, "_run_id", 0) if getattr(self, "_ckpt", None) is not None else 0

    def adjoint(self, gphi, gpsi=None, ckpt=None):
        """Reverse sweep of the last :meth:`forward_ckpt` run for the seed
        (dL/dphi(T), dL/dpsi(T)); returns (dL/dphi(0), dL/dpsi(0), dL/dA). Leaves the
        context without a state."""
        ck = ckpt if ckpt is not None else self._ckpt
        nb = ctypes.c_size_t(0)
        self._chk(self.lib.pcpf_adjoint_bytes(self.ctx, self._ckpt_every, ctypes.byref(nb)))
        scratch = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        sp = (scratch.data_ptr() + 255) // 256 * 256
        gphi_t = self._field(gphi)
        gpsi_t = self._field(gpsi) if gpsi is not None else None
        gphi0 = self.empty()
        gpsi0 = self.empty()
        ga = ctypes.c_double(0.0)
        self._chk(self.lib.pcpf_adjoint(self.ctx, _ptr(ck), ctypes.c_void_p(sp),
                                        ctypes.c_size_t(nb.value), _ptr(gphi_t), _ptr(gpsi_t),
                                        _ptr(gphi0), _ptr(gpsi0), ctypes.byref(ga)))
        return gphi0, gpsi0, ga.value

    def adjoint_static(self, gphi, gpsi=None, ckpt=None):
        """:meth:`adjoint` with the library's static per-GPU scratch instead of caller
        memory (pcpf_adjoint_static: allocates nothing; the run's scratch must fit
        PCPF_ADJOINT_STATIC_BYTES). The output tensors are the caller's, as always."""
        ck = ckpt if ckpt is not None else self._ckpt
        gphi_t = self._field(gphi)
        gpsi_t = self._field(gpsi) if gpsi is not None else None
        gphi0 = self.empty()
        gpsi0 = self.empty()
        ga = ctypes.c_double(0.0)
        self._chk(self.lib.pcpf_adjoint_static(self.ctx, _ptr(ck), _ptr(gphi_t), _ptr(gpsi_t),
                                               _ptr(gphi0), _ptr(gpsi0), ctypes.byref(ga)))
        return gphi0, gpsi0, ga.value
