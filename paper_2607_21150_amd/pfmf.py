"""Thin ctypes binding of libpfmf.so (the C ABI in include/pfmf.h).

Argument marshalling only: every step of the operator runs in the library's HIP
kernels. Torch provides device memory and the current stream. Importing this
module does not load the library; the first call does, and it raises if the
library is missing (there is no fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpfmf.so")

PF_OK, PF_EINVAL, PF_EHIP, PF_ENOMEM, PF_EUNSUPPORTED, PF_ENONPHYSICAL, PF_ENOCONV = 0, -1, -2, -3, -4, -5, -6

EXPORTED = [
    "pf_setup_mesh", "pf_sizes", "pf_set_params", "pf_apply_residual", "pf_apply_jacobian",
    "pf_apply_adjoint", "pf_linearize", "pf_level_info", "pf_apply_jacobian_f32", "pf_prolong",
    "pf_restrict", "pf_level_diagonal", "pf_pmg_vcycle", "pf_check", "pf_destroy", "pf_last_error",
    "pf_set_pmg_levels", "pf_set_dirichlet", "pf_commit_state", "pf_newton_step", "pf_set_option",
    "pf_apply_jacobian_lin", "pf_set_branches", "pf_commit_state_branches", "pf_set_geometry",
    "pf_setup_mesh_table", "pf_apply_adjoint_noalloc",
]

# pf_set_option
PF_OPT_SCATTER = 1
PF_OPT_STORE_LIN64 = 2
SCATTER_MODES = {"auto": 0, "colour": 1, "brick_buffer": 2}

# face indices of pf_set_dirichlet and field bits
FACES = {"x0": 0, "x1": 1, "y0": 2, "y1": 3, "z0": 4, "z1": 5}
FIELD_BITS = {"ux": 1, "uy": 2, "uz": 4, "phi": 8}


class PfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pfmf error {code}: {msg}")
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("p", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double)]


class TableMeshDesc(C.Structure):
    _fields_ = [("p", C.c_int), ("n_elem", C.c_int64), ("n_nodes", C.c_int64)]


class PhaseDesc(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("Gc", C.c_double), ("sigma0", C.c_double),
                ("H", C.c_double), ("visc", C.c_double), ("plastic", C.c_int),
                ("sigma_inf", C.c_double), ("voce_beta", C.c_double)]


class BranchDesc(C.Structure):
    _fields_ = [("kind", C.c_int), ("E", C.c_double), ("nu", C.c_double), ("eta_d", C.c_double),
                ("sigma0", C.c_double), ("H", C.c_double), ("visc", C.c_double), ("sigma_inf", C.c_double),
                ("voce_beta", C.c_double)]


# pf_branch kinds
PF_BRANCH_NONE, PF_BRANCH_HOOKE, PF_BRANCH_MAXWELL, PF_BRANCH_PRANDTL = 0, 1, 2, 3
PF_MAX_EXTRA_BRANCHES = 2


class FractureDesc(C.Structure):
    _fields_ = [("l0", C.c_double), ("eta", C.c_double), ("zeta", C.c_double), ("dt", C.c_double),
                ("s_phi", C.c_double), ("at", C.c_int)]


class PmgOpts(C.Structure):
    _fields_ = [("cheb_degree", C.c_int), ("coarse_p", C.c_int), ("coarse_sweeps", C.c_int),
                ("reserved", C.c_int)]


# pf_newton_opts.krylov
PF_KRYLOV_FGMRES, PF_KRYLOV_CG = 0, 1
KRYLOV = {"fgmres": PF_KRYLOV_FGMRES, "cg": PF_KRYLOV_CG}


class NewtonOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("restart", C.c_int), ("max_iters", C.c_int), ("cheb_degree", C.c_int),
                ("coarse_sweeps", C.c_int), ("krylov", C.c_int), ("reserved", C.c_int * 2)]


class NewtonStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("res0", C.c_double), ("res_lin", C.c_double),
                ("res_true", C.c_double), ("t_linearize_ms", C.c_double), ("t_total_ms", C.c_double),
                ("refinements", C.c_int), ("krylov", C.c_int), ("breakdown", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load():
    """Load libpfmf.so and declare its signatures (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or python -m paper_2607_21150_amd.build")
    L = C.CDLL(LIB_PATH)
    vp, i64p = C.c_void_p, C.POINTER(C.c_int64)
    L.pf_setup_mesh.argtypes = [C.POINTER(MeshDesc), C.POINTER(PhaseDesc), C.c_int, C.POINTER(FractureDesc),
                                vp, vp, vp, vp, C.POINTER(vp)]
    L.pf_setup_mesh_table.argtypes = [C.POINTER(TableMeshDesc), vp, vp, C.POINTER(PhaseDesc), C.c_int,
                                      C.POINTER(FractureDesc), vp, vp, vp, vp, C.POINTER(vp)]
    L.pf_sizes.argtypes = [vp, i64p, i64p, i64p]
    L.pf_set_params.argtypes = [vp, vp, vp]
    L.pf_apply_residual.argtypes = [vp, vp, vp, vp]
    L.pf_apply_jacobian.argtypes = [vp, vp, vp, vp, vp]
    L.pf_apply_adjoint.argtypes = [vp, vp, vp, vp, vp, vp]
    L.pf_apply_adjoint_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
    L.pf_linearize.argtypes = [vp, vp, vp]
    L.pf_level_info.argtypes = [vp, C.c_int, C.POINTER(C.c_int), i64p]
    L.pf_apply_jacobian_f32.argtypes = [vp, C.c_int, vp, vp, vp]
    L.pf_prolong.argtypes = [vp, C.c_int, vp, vp, vp]
    L.pf_restrict.argtypes = [vp, C.c_int, vp, vp, vp]
    L.pf_level_diagonal.argtypes = [vp, C.c_int, vp, vp]
    L.pf_pmg_vcycle.argtypes = [vp, vp, vp, C.POINTER(PmgOpts), vp]
    L.pf_set_pmg_levels.argtypes = [vp, vp, C.c_int]
    L.pf_set_dirichlet.argtypes = [vp, vp]
    L.pf_commit_state.argtypes = [vp, vp, vp, vp]
    L.pf_newton_step.argtypes = [vp, vp, C.POINTER(NewtonOpts), C.POINTER(NewtonStats), vp]
    L.pf_set_option.argtypes = [vp, C.c_int, C.c_int]
    L.pf_apply_jacobian_lin.argtypes = [vp, vp, vp, vp]
    L.pf_set_branches.argtypes = [vp, vp, C.c_int, vp]
    L.pf_commit_state_branches.argtypes = [vp, vp, vp, vp, vp]
    L.pf_set_geometry.argtypes = [vp, vp, vp]
    L.pf_check.argtypes = [vp]
    L.pf_destroy.argtypes = [vp]
    L.pf_destroy.restype = None
    L.pf_last_error.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("pf_destroy", "pf_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(code):
    if code != PF_OK:
        msg = load().pf_last_error().decode()
        raise PfError(code, msg)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _req(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise PfError(PF_EINVAL, f"{name} must be a device tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise PfError(PF_EINVAL, f"{name}: expected contiguous {dtype} {tuple(shape)}, "
                                 f"got {t.dtype} {tuple(t.shape)}")
    return t


class Context:
    """One operator context (pf_ctx). Holds references to the device state tensors."""

    def __init__(self, mesh, phases, fracture, qp_phase, qp_state, phi_n, stream=None, conn=None, X=None):
        """mesh: a box (pf_setup_mesh), or with ``conn`` (device int32 [n_elem][(p+1)^3], kept
        referenced) and ``X`` (device float64 [3][n_nodes]) a mesh given by its element table
        (pf_setup_mesh_table)."""
        L = load()
        self._phases = list(phases)
        arr = (PhaseDesc * len(phases))(*[PhaseDesc(p.E, p.nu, p.Gc, p.sigma0, p.H, p.visc, int(p.plastic),
                                                                 getattr(p, "sigma_inf", 0.0),
                                                                 getattr(p, "voce_beta", 0.0))
                                          for p in phases])
        fd = FractureDesc(fracture.l0, fracture.eta, fracture.zeta, fracture.dt, fracture.s_phi, int(fracture.at))
        self.n_nodes = mesh.n_nodes
        self.n_q = mesh.n_q
        self.mesh = mesh
        self.qp_phase = _req(qp_phase, torch.uint8, (mesh.n_q,), "qp_phase")
        self.qp_state = _req(qp_state, torch.float64, (8, mesh.n_q), "qp_state")
        self.phi_n = _req(phi_n, torch.float64, (mesh.n_nodes,), "phi_n")
        h = C.c_void_p()
        if conn is None:
            md = MeshDesc(mesh.p, mesh.nx, mesh.ny, mesh.nz, mesh.lx, mesh.ly, mesh.lz)
            _check(L.pf_setup_mesh(C.byref(md), arr, len(phases), C.byref(fd), _ptr(self.qp_phase),
                                   _ptr(self.qp_state), _ptr(self.phi_n), _stream(stream), C.byref(h)))
            self.conn = None
        else:
            P3 = (mesh.p + 1) ** 3
            self.conn = _req(conn, torch.int32, (mesh.n_elem, P3), "conn")
            X = _req(X, torch.float64, (3, mesh.n_nodes), "X")
            md = TableMeshDesc(mesh.p, mesh.n_elem, mesh.n_nodes)
            _check(L.pf_setup_mesh_table(C.byref(md), _ptr(self.conn), _ptr(X), arr, len(phases), C.byref(fd),
                                         _ptr(self.qp_phase), _ptr(self.qp_state), _ptr(self.phi_n),
                                         _stream(stream), C.byref(h)))
        self._h = h
        self.n_phases = len(phases)
        self.xstate = None

    @classmethod
    def from_inputs(cls, d, device="cuda"):
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        if d.get("conn") is not None:
            return cls(d["mesh"], d["phases"], d["fracture"], t(d["phase"], torch.uint8),
                       t(d["state"], torch.float64), t(d["phi_n"], torch.float64),
                       conn=t(d["conn"], torch.int32), X=t(d["X"], torch.float64))
        ctx = cls(d["mesh"], d["phases"], d["fracture"], t(d["phase"], torch.uint8),
                  t(d["state"], torch.float64), t(d["phi_n"], torch.float64))
        if d.get("branches"):
            ctx.set_branches(d["branches"], t(d["xstate"], torch.float64))
        if d.get("X") is not None:
            ctx.set_geometry(t(d["X"], torch.float64))
        return ctx

    def close(self):
        if getattr(self, "_h", None):
            load().pf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- C ABI calls (same names)
    def sizes(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(load().pf_sizes(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def set_branches(self, branches, xstate):
        """pf_set_branches: branches = per phase a list of n_extra branch descriptions
        (kind, E, nu, eta_d, sigma0, H, visc, sigma_inf, voce_beta); xstate = device
        float64 [7*n_extra][n_q], kept referenced. branches = None detaches."""
        if not branches:
            _check(load().pf_set_branches(self._h, None, 0, None))
            self.xstate = None
            return
        n_extra = len(branches[0])
        if len(branches) != self.n_phases or any(len(b) != n_extra for b in branches):
            raise PfError(PF_EINVAL, "branches: one list of equal length per phase")
        flat = [b for row in branches for b in row]
        arr = (BranchDesc * len(flat))(*[BranchDesc(int(b.kind), b.E, b.nu, b.eta_d, b.sigma0, b.H, b.visc,
                                                    b.sigma_inf, b.voce_beta) for b in flat])
        self.xstate = _req(xstate, torch.float64, (7 * n_extra, self.n_q), "xstate")
        _check(load().pf_set_branches(self._h, arr, n_extra, _ptr(self.xstate)))

    def set_geometry(self, X, stream=None):
        """pf_set_geometry: X = device float64 [3][n_nodes] node positions of a mapped mesh
        (read once, not kept); None returns to the box."""
        if X is None:
            _check(load().pf_set_geometry(self._h, None, _stream(stream)))
            return
        X = _req(X, torch.float64, (3, self.n_nodes), "X")
        _check(load().pf_set_geometry(self._h, _ptr(X), _stream(stream)))

    def set_params(self, params, stream=None):
        """pf_set_params: stream-ordered upload of the per-phase (Gc, sigma0, visc)."""
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(self.n_phases, 3))
        _check(load().pf_set_params(self._h, p.ctypes.data_as(C.c_void_p), _stream(stream)))

    def apply_residual(self, z, r=None, stream=None):
        _req(z, torch.float64, (4, self.n_nodes), "z")
        r = torch.empty_like(z) if r is None else _req(r, torch.float64, (4, self.n_nodes), "r")
        _check(load().pf_apply_residual(self._h, _ptr(z), _ptr(r), _stream(stream)))
        return r

    def apply_jacobian(self, z, dz, y=None, stream=None):
        _req(z, torch.float64, (4, self.n_nodes), "z")
        _req(dz, torch.float64, (4, self.n_nodes), "dz")
        y = torch.empty_like(z) if y is None else _req(y, torch.float64, (4, self.n_nodes), "y")
        _check(load().pf_apply_jacobian(self._h, _ptr(z), _ptr(dz), _ptr(y), _stream(stream)))
        return y

    def apply_adjoint(self, z, v, gz=None, gparams=None, stream=None):
        _req(z, torch.float64, (4, self.n_nodes), "z")
        _req(v, torch.float64, (4, self.n_nodes), "v")
        gz = torch.empty_like(z) if gz is None else _req(gz, torch.float64, (4, self.n_nodes), "gz")
        if gparams is None:
            gparams = torch.empty((self.n_phases, 3), dtype=torch.float64, device=z.device)
        _req(gparams, torch.float64, (self.n_phases, 3), "gparams")
        _check(load().pf_apply_adjoint(self._h, _ptr(z), _ptr(v), _ptr(gz), _ptr(gparams), _stream(stream)))
        return gz, gparams

    def apply_adjoint_noalloc(self, z, v, gz, gparams, stream=None):
        """pf_apply_adjoint_noalloc: the adjoint without any device allocation; gz and gparams
        must be given (the caller's memory)."""
        _req(z, torch.float64, (4, self.n_nodes), "z")
        _req(v, torch.float64, (4, self.n_nodes), "v")
        _req(gz, torch.float64, (4, self.n_nodes), "gz")
        _req(gparams, torch.float64, (self.n_phases, 3), "gparams")
        _check(load().pf_apply_adjoint_noalloc(self._h, _ptr(z), _ptr(v), _ptr(gz), _ptr(gparams), _stream(stream)))
        return gz, gparams

    def linearize(self, z, stream=None):
        _req(z, torch.float64, (4, self.n_nodes), "z")
        _check(load().pf_linearize(self._h, _ptr(z), _stream(stream)))

    def level_info(self, level):
        p, n = C.c_int(), C.c_int64()
        _check(load().pf_level_info(self._h, int(level), C.byref(p), C.byref(n)))
        return p.value, n.value

    def apply_jacobian_f32(self, level, dz, y=None, stream=None):
        _, n = self.level_info(level)
        _req(dz, torch.float32, (4, n), "dz")
        y = torch.empty_like(dz) if y is None else _req(y, torch.float32, (4, n), "y")
        _check(load().pf_apply_jacobian_f32(self._h, int(level), _ptr(dz), _ptr(y), _stream(stream)))
        return y

    def apply_jacobian_lin(self, dz, y=None, stream=None):
        """FP64 Jacobian at the last linearisation point, from the stored FP64 record."""
        _req(dz, torch.float64, (4, self.n_nodes), "dz")
        y = torch.empty_like(dz) if y is None else _req(y, torch.float64, (4, self.n_nodes), "y")
        _check(load().pf_apply_jacobian_lin(self._h, _ptr(dz), _ptr(y), _stream(stream)))
        return y

    def set_store_lin64(self, on):
        _check(load().pf_set_option(self._h, PF_OPT_STORE_LIN64, int(bool(on))))

    def prolong(self, level, xc, xf=None, stream=None):
        _, nf = self.level_info(level)
        _, nc = self.level_info(level + 1)
        _req(xc, torch.float32, (4, nc), "xc")
        xf = torch.empty((4, nf), dtype=torch.float32, device=xc.device) if xf is None else xf
        _check(load().pf_prolong(self._h, int(level), _ptr(xc), _ptr(xf), _stream(stream)))
        return xf

    def restrict(self, level, rf, rc=None, stream=None):
        _, nf = self.level_info(level)
        _, nc = self.level_info(level + 1)
        _req(rf, torch.float32, (4, nf), "rf")
        rc = torch.empty((4, nc), dtype=torch.float32, device=rf.device) if rc is None else rc
        _check(load().pf_restrict(self._h, int(level), _ptr(rf), _ptr(rc), _stream(stream)))
        return rc

    def level_diagonal(self, level, stream=None):
        _, n = self.level_info(level)
        d = torch.empty((4, n), dtype=torch.float32, device="cuda")
        _check(load().pf_level_diagonal(self._h, int(level), _ptr(d), _stream(stream)))
        return d

    def pmg_vcycle(self, b, x=None, cheb_degree=3, coarse_p=1, coarse_sweeps=4, stream=None):
        _req(b, torch.float32, (4, self.n_nodes), "b")
        x = torch.empty_like(b) if x is None else _req(x, torch.float32, (4, self.n_nodes), "x")
        o = PmgOpts(cheb_degree, coarse_p, coarse_sweeps, 0)
        _check(load().pf_pmg_vcycle(self._h, _ptr(b), _ptr(x), C.byref(o), _stream(stream)))
        return x

    def set_pmg_levels(self, orders):
        """Multigrid level orders, fine first (e.g. [4, 2, 1]); [] restores the default."""
        a = (C.c_int * max(len(orders), 1))(*orders)
        _check(load().pf_set_pmg_levels(self._h, C.cast(a, C.c_void_p), len(orders)))

    def set_dirichlet(self, faces):
        """faces: dict face name ('x0', 'x1', ...) -> iterable of field names ('ux', 'uy', 'uz', 'phi')."""
        arr = (C.c_uint32 * 6)()
        for face, fields in faces.items():
            arr[FACES[face]] = sum(FIELD_BITS[f] for f in fields)
        _check(load().pf_set_dirichlet(self._h, C.cast(arr, C.c_void_p)))

    def set_scatter(self, mode):
        """Scatter-add of the order-2/3 FP64 applies: 'auto', 'colour' or 'brick_buffer'."""
        _check(load().pf_set_option(self._h, PF_OPT_SCATTER, SCATTER_MODES[mode]))

    def commit_state(self, z, out=None, stream=None):
        _req(z, torch.float64, (4, self.n_nodes), "z")
        if out is None:
            out = torch.empty((8, self.n_q), dtype=torch.float64, device=z.device)
        _req(out, torch.float64, (8, self.n_q), "state_out")
        _check(load().pf_commit_state(self._h, _ptr(z), _ptr(out), _stream(stream)))
        return out

    def commit_state_branches(self, z, out=None, xout=None, stream=None):
        """pf_commit_state_branches: (state [8][n_q], extra branches' states [7*n_extra][n_q])."""
        _req(z, torch.float64, (4, self.n_nodes), "z")
        if self.xstate is None:
            raise PfError(PF_EINVAL, "no extra branch attached")
        if out is None:
            out = torch.empty((8, self.n_q), dtype=torch.float64, device=z.device)
        if xout is None:
            xout = torch.empty_like(self.xstate)
        _req(out, torch.float64, (8, self.n_q), "state_out")
        _req(xout, torch.float64, tuple(self.xstate.shape), "xstate_out")
        _check(load().pf_commit_state_branches(self._h, _ptr(z), _ptr(out), _ptr(xout), _stream(stream)))
        return out, xout

    def newton_step(self, z, rtol=1e-8, restart=30, max_iters=300, cheb_degree=3, coarse_sweeps=32,
                    stream=None, raise_on_noconv=True, krylov="fgmres"):
        """One Newton update of z in place; returns the solver report as a dict.
        krylov: 'fgmres' (default) or 'cg'."""
        _req(z, torch.float64, (4, self.n_nodes), "z")
        o = NewtonOpts(rtol, restart, max_iters, cheb_degree, coarse_sweeps, KRYLOV[krylov])
        st = NewtonStats()
        code = load().pf_newton_step(self._h, _ptr(z), C.byref(o), C.byref(st), _stream(stream))
        if code != PF_OK and not (code == PF_ENOCONV and not raise_on_noconv):
            _check(code)
        return st.as_dict()

    def check(self):
        _check(load().pf_check(self._h))


class PhaseFieldResidual(torch.autograd.Function):
    """r = R(z; params) as a differentiable torch op on the device.

    forward(z, params, op): ``z`` is the [4][n_nodes] FP64 device solution, ``params`` the
    [n_phases][3] per-phase (Gc, sigma0, visc) tensor, ``op`` a ``Context``. The context's
    parameters are set to ``params`` (they stay set after the call).
    backward(v): the hand-written adjoint kernel returns J(z)^T v and the per-phase partials
    dot(v, dR/d(Gc, sigma0, visc)); the pointwise linearisation is recomputed from z and the
    state, nothing is stored between forward and backward. Residual and its transposed
    linearisation follow the matrix-free residual and Jacobian of Section 4.
    """

    @staticmethod
    def forward(ctx, z, params, op):
        op.set_params(params.detach().to("cpu", torch.float64).numpy())
        r = op.apply_residual(z.detach().contiguous())
        ctx.save_for_backward(z, params)
        ctx.op = op
        return r

    @staticmethod
    def backward(ctx, v):
        z, params = ctx.saved_tensors
        op = ctx.op
        op.set_params(params.detach().to("cpu", torch.float64).numpy())
        gz, gp = op.apply_adjoint(z.detach().contiguous(), v.detach().to(torch.float64).contiguous())
        return gz, gp.to(device=params.device, dtype=params.dtype), None


def phase_field_residual(z, params, op):
    """Functional form of ``PhaseFieldResidual``."""
    return PhaseFieldResidual.apply(z, params, op)
