"""ctypes wrapper of the CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark. It builds the oracle with gcc on demand and
shares nothing with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"]
        subprocess.check_call(cmd, cwd=HERE)
        os.replace(tmp, LIB)
    return LIB


class OrMesh(C.Structure):
    _fields_ = [("p", C.c_int), ("q", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double), ("X", C.c_void_p),
                ("conn", C.c_void_p), ("n_elem", C.c_int64), ("n_nodes", C.c_int64)]


class OrPhase(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("Gc", C.c_double), ("sigma0", C.c_double),
                ("H", C.c_double), ("visc", C.c_double), ("plastic", C.c_int),
                ("sigma_inf", C.c_double), ("voce_beta", C.c_double)]


class OrBranch(C.Structure):
    _fields_ = [("kind", C.c_int), ("E", C.c_double), ("nu", C.c_double), ("eta_d", C.c_double),
                ("sigma0", C.c_double), ("H", C.c_double), ("visc", C.c_double), ("sigma_inf", C.c_double),
                ("voce_beta", C.c_double)]


MAX_EXTRA = 2


class OrFrac(C.Structure):
    _fields_ = [("l0", C.c_double), ("eta", C.c_double), ("zeta", C.c_double), ("dt", C.c_double),
                ("s_phi", C.c_double), ("at", C.c_int)]


class OrQpOut(C.Structure):
    _fields_ = [("P", C.c_double * 9), ("f0", C.c_double), ("f1", C.c_double * 3), ("tau", C.c_double * 6),
                ("beta", C.c_double * 3), ("eps", C.c_double * 3), ("theta", C.c_double), ("q", C.c_double),
                ("dgamma", C.c_double), ("c", C.c_double), ("psi_plus", C.c_double), ("H", C.c_double),
                ("L", C.c_double), ("g", C.c_double), ("plastic_active", C.c_int), ("nonphysical", C.c_int)]


_lib = None
_D = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        L.or_gauss.argtypes = [C.c_int, _D, _D]
        L.or_gll.argtypes = [C.c_int, _D]
        L.or_qf_residual.argtypes = [C.POINTER(OrPhase), C.POINTER(OrFrac), _D, C.c_double, _D, C.c_double,
                                     _D, C.POINTER(OrQpOut)]
        L.or_qf_jacobian.argtypes = [C.POINTER(OrPhase), C.POINTER(OrFrac), _D, C.c_double, _D, C.c_double,
                                     _D, _D, C.c_double, _D, _D, _D, _D]
        L.or_qf_param_partials.argtypes = [C.POINTER(OrPhase), C.POINTER(OrFrac), _D, C.c_double, _D,
                                           C.c_double, _D, _D, _D, _D]
        L.or_qf_residual_mb.argtypes = [C.POINTER(OrPhase), C.POINTER(OrBranch), C.c_int, C.POINTER(OrFrac), _D,
                                        C.c_double, _D, C.c_double, _D, _D, C.POINTER(OrQpOut)]
        L.or_qf_jacobian_mb.argtypes = [C.POINTER(OrPhase), C.POINTER(OrBranch), C.c_int, C.POINTER(OrFrac), _D,
                                        C.c_double, _D, C.c_double, _D, _D, _D, C.c_double, _D, _D, _D, _D]
        common = [C.POINTER(OrMesh), C.POINTER(OrPhase), C.c_int, C.POINTER(OrBranch), C.c_int,
                  C.POINTER(OrFrac), C.c_void_p, _D, _D, _D, _D]
        L.or_residual.argtypes = common + [_D, C.c_void_p, C.c_int64]
        L.or_jacobian.argtypes = common + [_D, _D, C.c_void_p, C.c_int64]
        L.or_adjoint.argtypes = common + [_D, _D, _D, C.c_void_p, C.c_int64]
        L.or_element_jacobian.argtypes = common + [C.c_int64, _D]
        L.or_qf_commit.argtypes = [C.POINTER(OrPhase), C.POINTER(OrFrac), _D, C.c_double, _D, _D]
        L.or_commit_state.argtypes = [C.POINTER(OrMesh), C.POINTER(OrPhase), C.c_int, C.POINTER(OrFrac),
                                      C.c_void_p, _D, _D, _D]
        L.or_commit_state.restype = C.c_int
        L.or_qf_commit_mb.argtypes = [C.POINTER(OrPhase), C.POINTER(OrBranch), C.c_int, C.POINTER(OrFrac), _D,
                                      C.c_double, _D, _D, _D, _D]
        L.or_commit_state_mb.argtypes = [C.POINTER(OrMesh), C.POINTER(OrPhase), C.c_int, C.POINTER(OrBranch),
                                         C.c_int, C.POINTER(OrFrac), C.c_void_p, _D, _D, _D, _D, _D]
        L.or_commit_state_mb.restype = C.c_int
        for f in ("or_residual", "or_jacobian", "or_adjoint", "or_element_jacobian"):
            getattr(L, f).restype = C.c_int
        L.or_num_threads.restype = C.c_int
        L.or_log_divdiff.argtypes = [C.c_double, C.c_double]
        L.or_log_divdiff.restype = C.c_double
        L.or_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def mesh_struct(mesh, q=None, X=None, conn=None):
    """X: node positions [3][n_nodes] (float64, C-contiguous, kept alive by the caller) or None.
    conn: element-to-node table int32 [n_elem][(p+1)^3] (kept alive by the caller) of a mesh
    with a table restriction (needs X), or None for the box lattice."""
    q = q if q is not None else mesh.p + 1
    Xp = X.ctypes.data_as(C.c_void_p) if X is not None else None
    if conn is not None:
        return OrMesh(mesh.p, q, 1, 1, 1, 1.0, 1.0, 1.0, Xp, conn.ctypes.data_as(C.c_void_p),
                      int(conn.shape[0]), int(mesh.n_nodes))
    return OrMesh(mesh.p, q, mesh.nx, mesh.ny, mesh.nz, mesh.lx, mesh.ly, mesh.lz, Xp, None, 0, 0)


def phase_struct(ph):
    return OrPhase(ph.E, ph.nu, ph.Gc, ph.sigma0, ph.H, ph.visc, int(ph.plastic),
                   getattr(ph, "sigma_inf", 0.0), getattr(ph, "voce_beta", 0.0))


def phases_array(phases):
    arr = (OrPhase * len(phases))()
    for i, ph in enumerate(phases):
        arr[i] = phase_struct(ph)
    return arr


def branch_struct(b):
    """b: inputs.Branch-like (kind, E, nu, eta_d, sigma0, H, visc, sigma_inf, voce_beta) or None."""
    if b is None:
        return OrBranch(0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    return OrBranch(int(b.kind), b.E, b.nu, b.eta_d, b.sigma0, b.H, b.visc, b.sigma_inf, b.voce_beta)


def branches_array(branches):
    """branches: list over phases of lists (length n_extra) of branches; -> (array, n_extra)."""
    if not branches:
        return None, 0
    n_extra = len(branches[0])
    assert all(len(b) == n_extra for b in branches) and 0 <= n_extra <= MAX_EXTRA
    arr = (OrBranch * max(1, len(branches) * n_extra))()
    for i, row in enumerate(branches):
        for j, b in enumerate(row):
            arr[i * n_extra + j] = branch_struct(b)
    return arr, n_extra


def frac_struct(fr):
    return OrFrac(fr.l0, fr.eta, fr.zeta, fr.dt, fr.s_phi, int(fr.at))


def gauss(n):
    x = np.zeros(n); w = np.zeros(n)
    lib().or_gauss(n, _p(x), _p(w))
    return x, w


def gll(n):
    x = np.zeros(n)
    lib().or_gll(n, _p(x))
    return x


def qf_residual(ph, fr, G, phi, gphi, phi_n, st):
    out = OrQpOut()
    G = _f64(np.reshape(G, 9)); gphi = _f64(gphi); st = _f64(st)
    lib().or_qf_residual(C.byref(phase_struct(ph)), C.byref(frac_struct(fr)), _p(G), float(phi), _p(gphi),
                         float(phi_n), _p(st), C.byref(out))
    return out


def qf_jacobian(ph, fr, G, phi, gphi, phi_n, st, dG, dphi, dgphi):
    G = _f64(np.reshape(G, 9)); gphi = _f64(gphi); st = _f64(st)
    dG = _f64(np.reshape(dG, 9)); dgphi = _f64(dgphi)
    dP = np.zeros(9); df0 = np.zeros(1); df1 = np.zeros(3)
    lib().or_qf_jacobian(C.byref(phase_struct(ph)), C.byref(frac_struct(fr)), _p(G), float(phi), _p(gphi),
                         float(phi_n), _p(st), _p(dG), float(dphi), _p(dgphi), _p(dP), _p(df0), _p(df1))
    return dP.reshape(3, 3), df0[0], df1


def qf_residual_mb(ph, xb, fr, G, phi, gphi, phi_n, st, xs):
    """Point with the extra branches xb (list, length n_extra) and their states xs[7*n_extra]."""
    out = OrQpOut()
    arr, n_extra = branches_array([xb])
    G = _f64(np.reshape(G, 9)); gphi = _f64(gphi); st = _f64(st); xs = _f64(np.reshape(xs, -1) if n_extra else np.zeros(1))
    lib().or_qf_residual_mb(C.byref(phase_struct(ph)), arr, n_extra, C.byref(frac_struct(fr)), _p(G), float(phi),
                            _p(gphi), float(phi_n), _p(st), _p(xs), C.byref(out))
    return out


def qf_jacobian_mb(ph, xb, fr, G, phi, gphi, phi_n, st, xs, dG, dphi, dgphi):
    arr, n_extra = branches_array([xb])
    G = _f64(np.reshape(G, 9)); gphi = _f64(gphi); st = _f64(st); xs = _f64(np.reshape(xs, -1) if n_extra else np.zeros(1))
    dG = _f64(np.reshape(dG, 9)); dgphi = _f64(dgphi)
    dP = np.zeros(9); df0 = np.zeros(1); df1 = np.zeros(3)
    lib().or_qf_jacobian_mb(C.byref(phase_struct(ph)), arr, n_extra, C.byref(frac_struct(fr)), _p(G), float(phi),
                            _p(gphi), float(phi_n), _p(st), _p(xs), _p(dG), float(dphi), _p(dgphi), _p(dP),
                            _p(df0), _p(df1))
    return dP.reshape(3, 3), df0[0], df1


def qf_param_partials(ph, fr, G, phi, gphi, phi_n, st):
    G = _f64(np.reshape(G, 9)); gphi = _f64(gphi); st = _f64(st)
    dP = np.zeros(27); df0 = np.zeros(3); df1 = np.zeros(9)
    lib().or_qf_param_partials(C.byref(phase_struct(ph)), C.byref(frac_struct(fr)), _p(G), float(phi),
                               _p(gphi), float(phi_n), _p(st), _p(dP), _p(df0), _p(df1))
    return dP.reshape(3, 3, 3), df0, df1.reshape(3, 3)


def qf_commit(ph, fr, G, phi, st):
    """New per-point state (D[6], ebar_p, H) after a converged step."""
    G = _f64(np.reshape(G, 9)); st = _f64(st)
    out = np.zeros(8)
    lib().or_qf_commit(C.byref(phase_struct(ph)), C.byref(frac_struct(fr)), _p(G), float(phi), _p(st), _p(out))
    return out


def qf_commit_mb(ph, xb, fr, G, phi, st, xs):
    """Commit of a point with extra branches: (new block state[8], new extra states[7*n_extra])."""
    arr, n_extra = branches_array([xb])
    G = _f64(np.reshape(G, 9)); st = _f64(st); xs = _f64(np.reshape(xs, -1))
    out = np.zeros(8); xout = np.zeros(max(7 * n_extra, 1))
    lib().or_qf_commit_mb(C.byref(phase_struct(ph)), arr, n_extra, C.byref(frac_struct(fr)), _p(G), float(phi),
                          _p(st), _p(xs), _p(out), _p(xout))
    return out, xout[:7 * n_extra]


class Oracle:
    """Oracle bound to one set of inputs (as produced by ``inputs.make_inputs``)."""

    def __init__(self, mesh, phases, fracture, phase, state, phi_n, branches=None, xstate=None, X=None, q=None,
                 conn=None):
        """X: node positions [3][n_nodes] of a mapped mesh (None: the box lattice); q: points
        per direction of the Gauss rule (None: p + 1; state and phase then hold n_elem*q^3
        points); conn: element-to-node table [n_elem][(p+1)^3] of a mesh with a table
        restriction (needs X)."""
        self.mesh = mesh
        self.X = _f64(X) if X is not None else None
        if self.X is not None:
            assert self.X.shape == (3, mesh.n_nodes)
        self.conn = np.ascontiguousarray(conn, dtype=np.int32) if conn is not None else None
        if self.conn is not None:
            assert self.X is not None and self.conn.shape[1] == (mesh.p + 1) ** 3
        self._m = mesh_struct(mesh, q=q, X=self.X, conn=self.conn)
        self._ph = phases_array(phases)
        self._nph = len(phases)
        self._fr = frac_struct(fracture)
        self.phase = np.ascontiguousarray(phase, dtype=np.uint8)
        self.state = _f64(state)
        self.phi_n = _f64(phi_n)
        self.set_branches(branches, xstate)

    @classmethod
    def from_inputs(cls, d):
        return cls(d["mesh"], d["phases"], d["fracture"], d["phase"], d["state"], d["phi_n"],
                   d.get("branches"), d.get("xstate"), d.get("X"), conn=d.get("conn"))

    def set_branches(self, branches, xstate):
        """Extra branches per phase (list over phases of lists of length n_extra) and their
        states [7*n_extra][n_q]; None detaches."""
        self._xbr, self._nx = branches_array(branches)
        if self._nx:
            assert len(branches) == self._nph
            self.xstate = _f64(xstate)
            assert self.xstate.shape == (7 * self._nx, self.state.shape[1])
        else:
            self.xstate = np.zeros(1)

    def set_phases(self, phases):
        self._ph = phases_array(phases)
        self._nph = len(phases)

    def _elems(self, elems):
        if elems is None:
            return None, 0, None
        e = np.ascontiguousarray(elems, dtype=np.int32)
        return e.ctypes.data_as(C.c_void_p), len(e), e

    def _common(self):
        return (C.byref(self._m), self._ph, self._nph, self._xbr, self._nx, C.byref(self._fr),
                self.phase.ctypes.data_as(C.c_void_p), _p(self.state), _p(self.xstate), _p(self.phi_n))

    def residual(self, z, elems=None, check=True):
        z = _f64(z)
        r = np.zeros_like(z)
        ep, n, keep = self._elems(elems)
        rc = lib().or_residual(*self._common(), _p(z), _p(r), ep, n)
        if rc < 0 or (check and rc):
            raise RuntimeError(f"oracle residual failed: {rc}")
        return r

    def jacobian(self, z, dz, elems=None, check=True):
        z = _f64(z); dz = _f64(dz)
        y = np.zeros_like(z)
        ep, n, keep = self._elems(elems)
        rc = lib().or_jacobian(*self._common(), _p(z), _p(dz), _p(y), ep, n)
        if rc < 0 or (check and rc):
            raise RuntimeError(f"oracle jacobian failed: {rc}")
        return y

    def adjoint(self, z, v, elems=None, check=True):
        z = _f64(z); v = _f64(v)
        g = np.zeros_like(z)
        gp = np.zeros(self._nph * 3)
        ep, n, keep = self._elems(elems)
        rc = lib().or_adjoint(*self._common(), _p(z), _p(v), _p(g), _p(gp), ep, n)
        if rc < 0 or (check and rc):
            raise RuntimeError(f"oracle adjoint failed: {rc}")
        return g, gp.reshape(self._nph, 3)

    def commit_state(self, z):
        """State [8][n_q] after a converged step at z (exponential-map update); with extra
        branches the pair (state, xstate)."""
        z = _f64(z)
        out = np.zeros_like(self.state)
        if not self._nx:
            rc = lib().or_commit_state(C.byref(self._m), self._ph, self._nph, C.byref(self._fr),
                                       self.phase.ctypes.data_as(C.c_void_p), _p(self.state), _p(z), _p(out))
            if rc < 0:
                raise RuntimeError("oracle commit failed")
            return out
        xout = np.zeros_like(self.xstate)
        rc = lib().or_commit_state_mb(C.byref(self._m), self._ph, self._nph, self._xbr, self._nx, C.byref(self._fr),
                                      self.phase.ctypes.data_as(C.c_void_p), _p(self.state), _p(self.xstate), _p(z),
                                      _p(out), _p(xout))
        if rc < 0:
            raise RuntimeError("oracle commit failed")
        return out, xout

    def element_jacobian(self, z, e):
        z = _f64(z)
        nd = 4 * (self.mesh.p + 1) ** 3
        K = np.zeros((nd, nd))
        rc = lib().or_element_jacobian(*self._common(), _p(z), int(e), _p(K))
        if rc < 0:
            raise RuntimeError("oracle element jacobian failed")
        return K

    def element_nodes(self, e):
        if self.conn is not None:
            return self.conn[e].astype(np.int64)
        m = self.mesh
        P = m.p + 1
        nx1, ny1, _ = m.node_dims
        ex, ey, ez = e % m.nx, (e // m.nx) % m.ny, e // (m.nx * m.ny)
        a = np.arange(P)
        gx = ex * m.p + a[None, None, :]
        gy = ey * m.p + a[None, :, None]
        gz = ez * m.p + a[:, None, None]
        return (gx + nx1 * (gy + ny1 * gz)).reshape(-1)


def log_divdiff(bi_m1: float, bj_m1: float) -> float:
    """(ln b_i - ln b_j) / (b_i - b_j) with b = 1 + beta: the oracle's off-diagonal tangent factor."""
    return float(lib().or_log_divdiff(float(bi_m1), float(bj_m1)))


def num_threads():
    return lib().or_num_threads()


def set_num_threads(n):
    lib().or_set_num_threads(int(n))
