"""Seeded synthetic inputs for the coupled displacement / phase-field operator.

This module only *draws* inputs: mesh descriptors, particle microstructures,
nodal fields, per-quadrature-point state and probe directions. It holds none of
the operator's arithmetic (no kinematics, return mapping, basis contractions or
assembly), so both the CPU oracle and the HIP library can be fed from it.

Data layout shared by every consumer (an interface convention, not arithmetic):

* structured box of ``nx*ny*nz`` hexahedra of order ``p``; nodes sit at the
  Gauss-Lobatto-Legendre (GLL) points of each element, numbered lexicographically
  x-fastest over the global ``(p*nx+1) x (p*ny+1) x (p*nz+1)`` lattice;
* solution ``z`` is SoA ``[4][n_nodes]`` float64: ``u_x, u_y, u_z, phi``;
* quadrature is tensor Gauss-Legendre with ``Q = p+1`` points per direction;
  quadrature points are numbered element-major (``e = ex + nx*(ey + ny*ez)``)
  and x-fastest inside the element: ``qp = e*Q^3 + qx + Q*(qy + Q*qz)``;
* per-point state is SoA ``[8][n_q]`` float64: ``D`` (6, Voigt order
  xx, yy, zz, yz, xz, xy) with ``D = C^{in,-1}_n - I``, the accumulated plastic
  strain, and the history field ``H_n``; the phase id is ``uint8[n_q]``
  (0 = matrix, 1 = particle);
* with extra branches in parallel (variant ``ex3``), their state is SoA
  ``[7*n_extra][n_q]`` float64: per branch ``D`` (6) and its accumulated plastic
  strain.

Units are mm, MPa, s and N/mm (so G_c in N/mm = kJ/m^2).

Workload recipes (the paper's microstructures and meshes are not available;
these structured particle-matrix cubes stand in for them):

* ``C1`` Q2 on 4^3 elements, 6 spheres with radius U[0.1, 0.2] mm;
* ``C2`` Q2 on 32^3, 40 spheres at 30 % volume fraction;
* ``C3`` Q3 on 48^3, 150 spheres at 30 %;
* ``C4`` the adjoint case, same mesh as C2;
* ``C5`` Q4 on 40^3, 200 spheres at 35 %.

Radii are drawn U[0.03, 0.08] mm for C2-C5 and then scaled by one common
factor (bisection) until the union of spheres covers the target fraction of
a probe lattice, because that radius range alone cannot reach 30 %.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Mesh", "UMesh", "Phase", "Branch", "Fracture", "Config", "CONFIGS", "make_config",
    "make_inputs", "unstructured", "gll_points", "gauss_points", "default_phases",
    "default_fracture",
]

SEED_BASE = 21150
# one independent random stream per purpose
(STREAM_SPHERES, STREAM_PHI, STREAM_SINES, STREAM_STATE, STREAM_DIR, STREAM_COT, STREAM_XSTATE,
 STREAM_UNSTRUCT) = range(8)

# kinds of extra branches in parallel with a phase's block
BRANCH_NONE, BRANCH_HOOKE, BRANCH_MAXWELL, BRANCH_PRANDTL = 0, 1, 2, 3


@dataclasses.dataclass(frozen=True)
class Mesh:
    p: int
    nx: int
    ny: int
    nz: int
    lx: float = 1.0
    ly: float = 1.0
    lz: float = 1.0

    @property
    def q(self) -> int:
        return self.p + 1

    @property
    def node_dims(self):
        return (self.p * self.nx + 1, self.p * self.ny + 1, self.p * self.nz + 1)

    @property
    def n_nodes(self) -> int:
        a, b, c = self.node_dims
        return a * b * c

    @property
    def n_elem(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_q(self) -> int:
        return self.n_elem * self.q ** 3

    @property
    def n_dof(self) -> int:
        return 4 * self.n_nodes


@dataclasses.dataclass(frozen=True)
class UMesh:
    """Hexahedral mesh given by a table restriction: ``n_elem`` elements of order ``p``
    whose ``(p+1)^3`` nodes are listed, per element, in the element's own reference
    coordinates (local node ``a = ax + P*(ay + P*az)``), over ``n_nodes`` nodes with
    arbitrary numbering. Quadrature points stay element-major with ``Q = p+1`` Gauss
    points per direction in the element's reference coordinates. ``box`` is the lattice
    mesh the synthetic table was cut from (its size and extent)."""
    p: int
    n_elem: int
    n_nodes: int
    box: Mesh

    @property
    def q(self) -> int:
        return self.p + 1

    @property
    def n_q(self) -> int:
        return self.n_elem * self.q ** 3

    @property
    def n_dof(self) -> int:
        return 4 * self.n_nodes

    @property
    def lx(self) -> float:
        return self.box.lx


@dataclasses.dataclass(frozen=True)
class Phase:
    """Material of one phase: Hencky (Hooke) branch plus optional Prandtl branch."""
    E: float
    nu: float
    Gc: float
    sigma0: float = 0.0
    H: float = 0.0          # linear hardening modulus
    visc: float = 0.0       # overstress viscosity [s]
    plastic: bool = False
    sigma_inf: float = 0.0  # Voce saturation stress [MPa] (with voce_beta > 0)
    voce_beta: float = 0.0  # Voce rate; 0 = linear hardening


@dataclasses.dataclass(frozen=True)
class Branch:
    """Extra rheological branch in parallel with a phase's block: its own spring
    (E, nu), a Maxwell branch's deviatoric viscosity eta_d [MPa s], a Prandtl
    branch's hardening and overstress (as in Phase)."""
    kind: int
    E: float = 0.0
    nu: float = 0.0
    eta_d: float = 0.0
    sigma0: float = 0.0
    H: float = 0.0
    visc: float = 0.0
    sigma_inf: float = 0.0
    voce_beta: float = 0.0


@dataclasses.dataclass(frozen=True)
class Fracture:
    l0: float
    eta: float = 1e-3       # residual stiffness factor
    zeta: float = 1e-2      # damage viscosity [MPa s]
    dt: float = 1e-2        # time step [s]
    s_phi: float = 1.0      # global phase-field residual scale
    at: int = 1             # 1 = AT1, 2 = AT2


def default_phases():
    """Phase 0 = visco-elastoplastic matrix, phase 1 = elastic particle."""
    matrix = Phase(E=1000.0, nu=0.45, Gc=0.2, sigma0=10.0, H=100.0, visc=1e-2, plastic=True)
    particle = Phase(E=15000.0, nu=0.3, Gc=0.05)
    return [matrix, particle]


def voce_phases():
    """The default phases with Voce hardening on the matrix (saturation 30 MPa, rate 50)."""
    matrix, particle = default_phases()
    return [dataclasses.replace(matrix, sigma_inf=30.0, voce_beta=50.0), particle]


def ex3_phases():
    """The visco-elastoplastic matrix and the particle of the paper's third example
    (its material table, in MPa, MPa s and N/mm): matrix = perfectly plastic Prandtl
    block (E2 = 198 GPa, nu = 0.3, sigma0 = 500 MPa) in parallel with a Hooke spring
    (1 GPa, 0.3) and a Maxwell branch (1 GPa, 0.3, eta_d = 0.01 GPa s); particle =
    Hooke (400 GPa, 0.25). Returns (phases, branches[n_phases][2])."""
    matrix = Phase(E=198000.0, nu=0.3, Gc=0.8, sigma0=500.0, H=0.0, visc=0.0, plastic=True)
    particle = Phase(E=400000.0, nu=0.25, Gc=8.0)
    xb_matrix = [Branch(BRANCH_HOOKE, E=1000.0, nu=0.3), Branch(BRANCH_MAXWELL, E=1000.0, nu=0.3, eta_d=10.0)]
    xb_particle = [Branch(BRANCH_NONE), Branch(BRANCH_NONE)]
    return [matrix, particle], [xb_matrix, xb_particle]


def default_fracture(mesh: Mesh, phases, at: int = 1) -> Fracture:
    h = mesh.lx / mesh.nx
    l0 = 2.0 * h
    c0 = 8.0 / 3.0 if at == 1 else 2.0
    m = phases[0]
    s_phi = m.E * c0 / (2.0 * l0 * m.Gc)
    return Fracture(l0=l0, s_phi=s_phi, at=at)


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    cfg_id: int
    p: int
    n: int
    n_spheres: int
    r_lo: float
    r_hi: float
    vol_frac: Optional[float]


CONFIGS = {
    "C1": Config("C1", 1, 2, 4, 6, 0.1, 0.2, None),
    "C2": Config("C2", 2, 2, 32, 40, 0.03, 0.08, 0.30),
    "C3": Config("C3", 3, 3, 48, 150, 0.03, 0.08, 0.30),
    "C4": Config("C4", 4, 2, 32, 40, 0.03, 0.08, 0.30),
    "C5": Config("C5", 5, 4, 40, 200, 0.03, 0.08, 0.35),
}

VARIANT_E0 = {"base": 1e-3, "plastic": 2e-2, "compress": -1e-3, "voce": 2e-2, "ex3": 1e-2,
              "ex3_compress": -5e-3}


def make_config(name: str, p: Optional[int] = None, n: Optional[int] = None) -> Config:
    c = CONFIGS[name]
    if p is not None or n is not None:
        c = dataclasses.replace(c, p=p if p is not None else c.p, n=n if n is not None else c.n)
    return c


def _rng(cfg_id: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + 100 * cfg_id + stream))


def gll_points(p: int) -> np.ndarray:
    """GLL points on [-1, 1] (endpoints plus roots of P_p')."""
    if p == 1:
        return np.array([-1.0, 1.0])
    inner = np.polynomial.legendre.Legendre.basis(p).deriv().roots()
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def gauss_points(q: int) -> np.ndarray:
    return np.polynomial.legendre.leggauss(q)[0]


def _coords_1d(n: int, p: int, length: float, ref: np.ndarray) -> np.ndarray:
    """Physical coordinates of the points ``ref`` (on [-1,1]) of all n cells.

    For GLL nodes the shared end points are merged (size p*n+1); for interior
    points (Gauss) the result has size n*len(ref).
    """
    h = length / n
    loc = 0.5 * (ref + 1.0) * h
    if len(ref) == p + 1 and ref[0] == -1.0 and ref[-1] == 1.0:
        out = np.empty(p * n + 1)
        for e in range(n):
            out[p * e: p * e + p + 1] = e * h + loc
        out[-1] = length
        return out
    return (np.arange(n)[:, None] * h + loc[None, :]).reshape(-1)


def _spheres(cfg: Config, mesh: Mesh):
    rng = _rng(cfg.cfg_id, STREAM_SPHERES)
    centres = rng.uniform(0.0, 1.0, size=(cfg.n_spheres, 3)) * np.array([mesh.lx, mesh.ly, mesh.lz])
    radii = rng.uniform(cfg.r_lo, cfg.r_hi, size=cfg.n_spheres)
    if cfg.vol_frac is None:
        return centres, radii, 1.0
    # bisect a common radius scale on a probe lattice (cell centres, 96^3)
    m = 96
    g = (np.arange(m) + 0.5) / m
    probe = (g * mesh.lx, g * mesh.ly, g * mesh.lz)

    def frac(scale):
        return _union_mask(probe, centres, radii * scale).mean()

    lo, hi = 0.5, 8.0
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        if frac(mid) < cfg.vol_frac:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-4:
            break
    scale = 0.5 * (lo + hi)
    return centres, radii * scale, scale


def _union_mask(axes, centres, radii) -> np.ndarray:
    """Boolean [z][y][x] mask of lattice points inside any sphere."""
    xs, ys, zs = axes
    mask = np.zeros((len(zs), len(ys), len(xs)), dtype=bool)
    for c, r in zip(centres, radii):
        ix = np.nonzero(np.abs(xs - c[0]) <= r)[0]
        iy = np.nonzero(np.abs(ys - c[1]) <= r)[0]
        iz = np.nonzero(np.abs(zs - c[2]) <= r)[0]
        if len(ix) == 0 or len(iy) == 0 or len(iz) == 0:
            continue
        dx = (xs[ix] - c[0]) ** 2
        dy = (ys[iy] - c[1]) ** 2
        dz = (zs[iz] - c[2]) ** 2
        inside = (dz[:, None, None] + dy[None, :, None] + dx[None, None, :]) <= r * r
        sub = mask[iz[0]:iz[-1] + 1, iy[0]:iy[-1] + 1, ix[0]:ix[-1] + 1]
        sub |= inside
    return mask


def _grid_to_qp_order(grid: np.ndarray, mesh: Mesh) -> np.ndarray:
    """[z*Q+qz][y*Q+qy][x*Q+qx] lattice -> element-major qp ordering."""
    Q = mesh.q
    g = grid.reshape(mesh.nz, Q, mesh.ny, Q, mesh.nx, Q)
    g = g.transpose(0, 2, 4, 1, 3, 5)  # ez, ey, ex, qz, qy, qx
    return np.ascontiguousarray(g).reshape(-1)


def curved_nodes(mesh: Mesh, amp: float = 0.2):
    """Node positions of a curved mesh: the box's GLL lattice moved by
    amp * h * sin(2 pi x / lam) sin(2 pi y / lam) sin(2 pi z / lam) * (1, 0.7, -0.5) with
    lam = 4 h, so elements are curved at their own scale while every boundary face stays
    planar (the field vanishes there when the element count per side is even)."""
    gll = gll_points(mesh.p)
    X = _coords_1d(mesh.nx, mesh.p, mesh.lx, gll)
    Y = _coords_1d(mesh.ny, mesh.p, mesh.ly, gll)
    Z = _coords_1d(mesh.nz, mesh.p, mesh.lz, gll)
    h = mesh.lx / mesh.nx
    lam = 4.0 * h
    sx = np.sin(2 * math.pi * X / lam)
    sy = np.sin(2 * math.pi * Y / lam)
    sz = np.sin(2 * math.pi * Z / lam)
    bump = amp * h * sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    nz1, ny1, nx1 = len(Z), len(Y), len(X)
    out = np.empty((3, nz1, ny1, nx1))
    out[0] = X[None, None, :] + 1.0 * bump
    out[1] = Y[None, :, None] + 0.7 * bump
    out[2] = Z[:, None, None] - 0.5 * bump
    return out.reshape(3, -1)


def make_inputs(name: str = "C1", variant: str = "base", p: Optional[int] = None,
                n: Optional[int] = None, phases=None, at: int = 1, with_dir: bool = True,
                geometry: str = "box"):
    """Draw every input of one configuration.

    Returns a dict with ``mesh``, ``phases``, ``fracture``, ``z`` [4][n_nodes],
    ``phi_n`` [n_nodes], ``state`` [8][n_q], ``phase`` uint8[n_q],
    ``dz`` [4][n_nodes] (unit l2 norm), ``v_top`` (top-face u_z indicator) and
    ``v_rand`` [4][n_nodes] (unit l2 norm). The ``ex3`` variants add ``branches``
    (per phase, the extra branches) and ``xstate`` [7*n_extra][n_q]. ``geometry="curved"``
    adds ``X`` [3][n_nodes], the node positions of a curved mesh (see curved_nodes).
    """
    cfg = make_config(name, p, n)
    mesh = Mesh(cfg.p, cfg.n, cfg.n, cfg.n)
    branches = None
    if variant.startswith("ex3"):
        phases, branches = ex3_phases()
    elif phases is None:
        phases = voce_phases() if variant == "voce" else default_phases()
    frac = default_fracture(mesh, phases, at)
    e0 = VARIANT_E0[variant]
    P = mesh.p
    nx1, ny1, nz1 = mesh.node_dims
    gll = gll_points(P)
    X = _coords_1d(mesh.nx, P, mesh.lx, gll)
    Y = _coords_1d(mesh.ny, P, mesh.ly, gll)
    Z = _coords_1d(mesh.nz, P, mesh.lz, gll)

    # displacement: uniaxial strain along z plus a seeded sum of sines per component
    rng = _rng(cfg.cfg_id, STREAM_SINES)
    u = np.zeros((3, nz1, ny1, nx1))
    u[2] += e0 * Z[:, None, None]
    for comp in range(3):
        pert = np.zeros((nz1, ny1, nx1))
        for _ in range(4):
            k = rng.integers(1, 4, size=3)
            ph = rng.uniform(0.0, 2.0 * math.pi)
            sx = 2 * math.pi * k[0] * X
            sy = 2 * math.pi * k[1] * Y
            sz = 2 * math.pi * k[2] * Z
            pert += np.sin(sz[:, None, None] + sy[None, :, None] + sx[None, None, :] + ph)
        pert *= 1e-4 / np.abs(pert).max()
        u[comp] += pert

    # phase field: max over three seeds of 0.9 exp(-d^2 / l0^2)
    rng = _rng(cfg.cfg_id, STREAM_PHI)
    seeds = rng.uniform(0.0, 1.0, size=(3, 3)) * np.array([mesh.lx, mesh.ly, mesh.lz])
    phi = np.zeros((nz1, ny1, nx1))
    for s in seeds:
        d2 = ((Z - s[2]) ** 2)[:, None, None] + ((Y - s[1]) ** 2)[None, :, None] + ((X - s[0]) ** 2)[None, None, :]
        np.maximum(phi, 0.9 * np.exp(-d2 / frac.l0 ** 2), out=phi)

    z = np.empty((4, mesh.n_nodes))
    z[:3] = u.reshape(3, -1)
    z[3] = phi.reshape(-1)
    phi_n = 0.99 * z[3]

    # microstructure -> per-qp phase id
    centres, radii, scale = _spheres(cfg, mesh)
    gq = gauss_points(mesh.q)
    Xq = _coords_1d(mesh.nx, P, mesh.lx, gq)
    Yq = _coords_1d(mesh.ny, P, mesh.ly, gq)
    Zq = _coords_1d(mesh.nz, P, mesh.lz, gq)
    inside = _union_mask((Xq, Yq, Zq), centres, radii)
    phase = _grid_to_qp_order(inside, mesh).astype(np.uint8)

    # per-qp state (matrix only carries inelastic history)
    rng = _rng(cfg.cfg_id, STREAM_STATE)
    nq = mesh.n_q
    state = np.zeros((8, nq))
    ep = rng.uniform(-1e-4, 1e-4, size=(nq, 6))
    tr = (ep[:, 0] + ep[:, 1] + ep[:, 2]) / 3.0
    ep[:, :3] -= tr[:, None]
    # D = exp(-2 eps_p) - I (isochoric inelastic stretch, symmetric, no rotation)
    E = np.zeros((nq, 3, 3))
    E[:, 0, 0], E[:, 1, 1], E[:, 2, 2] = ep[:, 0], ep[:, 1], ep[:, 2]
    E[:, 1, 2] = E[:, 2, 1] = ep[:, 3]
    E[:, 0, 2] = E[:, 2, 0] = ep[:, 4]
    E[:, 0, 1] = E[:, 1, 0] = ep[:, 5]
    lam, V = np.linalg.eigh(E)
    Dm = np.einsum("qij,qj,qkj->qik", V, np.expm1(-2.0 * lam), V)
    del E, V, lam
    state[0], state[1], state[2] = Dm[:, 0, 0], Dm[:, 1, 1], Dm[:, 2, 2]
    state[3], state[4], state[5] = Dm[:, 1, 2], Dm[:, 0, 2], Dm[:, 0, 1]
    del Dm
    state[6] = rng.uniform(0.0, 1e-2, size=nq)
    psi_hat = []
    for ph in phases:
        mu = ph.E / (2.0 * (1.0 + ph.nu))
        kappa = ph.E / (3.0 * (1.0 - 2.0 * ph.nu))
        psi_hat.append(0.5 * (kappa + 4.0 * mu / 3.0) * e0 * e0)
    hmax = np.where(phase == 0, 2.0 * psi_hat[0], 2.0 * psi_hat[1 % len(phases)])
    state[7] = rng.uniform(0.0, 1.0, size=nq) * hmax
    part = phase != 0
    state[:7, part] = 0.0

    out = dict(mesh=mesh, phases=list(phases), fracture=frac, z=z, phi_n=phi_n,
               state=state, phase=phase, cfg=cfg, variant=variant, e0=e0,
               sphere_scale=scale, vol_frac=float(phase.mean()))
    if geometry == "curved":
        out["X"] = curved_nodes(mesh)
    elif geometry != "box":
        raise ValueError(f"geometry {geometry!r}")
    if branches is not None:
        # extra branches' states: an isochoric D per inelastic branch drawn like the
        # block's (accumulated plastic strain 0), zero in the particles
        n_extra = len(branches[0])
        rng = _rng(cfg.cfg_id, STREAM_XSTATE)
        xstate = np.zeros((7 * n_extra, nq))
        for j in range(n_extra):
            ep = rng.uniform(-1e-4, 1e-4, size=(nq, 6))
            tr = (ep[:, 0] + ep[:, 1] + ep[:, 2]) / 3.0
            ep[:, :3] -= tr[:, None]
            E = np.zeros((nq, 3, 3))
            E[:, 0, 0], E[:, 1, 1], E[:, 2, 2] = ep[:, 0], ep[:, 1], ep[:, 2]
            E[:, 1, 2] = E[:, 2, 1] = ep[:, 3]
            E[:, 0, 2] = E[:, 2, 0] = ep[:, 4]
            E[:, 0, 1] = E[:, 1, 0] = ep[:, 5]
            lam, V = np.linalg.eigh(E)
            Dm = np.einsum("qij,qj,qkj->qik", V, np.expm1(-2.0 * lam), V)
            del E, V, lam
            r = 7 * j
            xstate[r], xstate[r + 1], xstate[r + 2] = Dm[:, 0, 0], Dm[:, 1, 1], Dm[:, 2, 2]
            xstate[r + 3], xstate[r + 4], xstate[r + 5] = Dm[:, 1, 2], Dm[:, 0, 2], Dm[:, 0, 1]
            del Dm
        xstate[:, part] = 0.0
        out["branches"] = branches
        out["xstate"] = xstate
    if with_dir:
        rng = _rng(cfg.cfg_id, STREAM_DIR)
        dz = rng.standard_normal((4, mesh.n_nodes))
        dz /= np.linalg.norm(dz)
        out["dz"] = dz
        rng = _rng(cfg.cfg_id, STREAM_COT)
        vr = rng.standard_normal((4, mesh.n_nodes))
        vr /= np.linalg.norm(vr)
        out["v_rand"] = vr
        v_top = np.zeros((4, mesh.n_nodes))
        top = np.arange(mesh.n_nodes).reshape(nz1, ny1, nx1)[-1].reshape(-1)
        v_top[2, top] = 1.0
        out["v_top"] = v_top
    return out


def node_index(mesh: Mesh, ix, iy, iz):
    nx1, ny1, _ = mesh.node_dims
    return ix + nx1 * (iy + ny1 * iz)


def elements_touching_nodes(mesh: Mesh, nodes) -> np.ndarray:
    """Element ids whose closure contains any of ``nodes`` (for sampled checks)."""
    nx1, ny1, _ = mesh.node_dims
    nodes = np.asarray(nodes)
    ix = nodes % nx1
    iy = (nodes // nx1) % ny1
    iz = nodes // (nx1 * ny1)
    out = set()
    P = mesh.p
    for a, b, c in zip(ix, iy, iz):
        exs = {min(a // P, mesh.nx - 1)} | ({a // P - 1} if a % P == 0 and a > 0 else set())
        eys = {min(b // P, mesh.ny - 1)} | ({b // P - 1} if b % P == 0 and b > 0 else set())
        ezs = {min(c // P, mesh.nz - 1)} | ({c // P - 1} if c % P == 0 and c > 0 else set())
        for ex in exs:
            for ey in eys:
                for ez in ezs:
                    out.add(ex + mesh.nx * (ey + mesh.ny * ez))
    return np.array(sorted(out), dtype=np.int32)


def lattice_connectivity(mesh: Mesh) -> np.ndarray:
    """Element-to-node table [n_elem][P^3] of the box lattice (the numbering of this module)."""
    P = mesh.p + 1
    nx1, ny1, _ = mesh.node_dims
    e = np.arange(mesh.n_elem)
    ex, ey, ez = e % mesh.nx, (e // mesh.nx) % mesh.ny, e // (mesh.nx * mesh.ny)
    a = np.arange(P)
    az, ay, ax = np.meshgrid(a, a, a, indexing="ij")
    ax, ay, az = ax.reshape(-1), ay.reshape(-1), az.reshape(-1)
    gx = ex[:, None] * mesh.p + ax[None, :]
    gy = ey[:, None] * mesh.p + ay[None, :]
    gz = ez[:, None] * mesh.p + az[None, :]
    return (gx + nx1 * (gy + ny1 * gz)).astype(np.int64)


def cube_rotations():
    """The 24 proper rotations of the reference cube, as signed 3x3 permutation matrices."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3), dtype=np.int64)
            for i in range(3):
                R[i, perm[i]] = signs[i]
            if round(np.linalg.det(R)) == 1:
                out.append(R)
    return out


def rotated_local_index(R: np.ndarray, n: int) -> np.ndarray:
    """For a grid of n points per direction, symmetric about the cube's centre (GLL nodes,
    Gauss points): idx[a'] = the lattice-local index of the point R xi(a') (x fastest)."""
    c = 2 * np.arange(n) - (n - 1)
    cz, cy, cx = np.meshgrid(c, c, c, indexing="ij")
    C = np.stack([cx.reshape(-1), cy.reshape(-1), cz.reshape(-1)])
    il = (R @ C + (n - 1)) // 2
    return il[0] + n * (il[1] + n * il[2])


def unstructured(d, hole_radius: float = 0.0, node_order: str = "random", shuffle_elements: bool = True,
                 rotate: bool = True):
    """The inputs ``d`` of a box (or curved) lattice re-expressed on a mesh given by a table
    restriction (UMesh): elements whose centre lies within ``hole_radius`` of the axis
    x = lx/2, z = lz/2 are removed (a cylindrical hole, so node valences vary), every kept
    element gets one of the 24 proper cube rotations as its own local orientation (``rotate``),
    the elements are shuffled (``shuffle_elements``), and the nodes in use are renumbered:
    ``node_order`` "random" (a random permutation) or "first_touch" (order of first appearance
    in the element table, as a mesh generator's renumbering would give). Fields, state and
    phase ids are carried over unchanged by index maps (the physics is the same; only the
    numbering and the element orientation change). Adds ``conn`` int32 [n_elem][P^3], ``X``
    [3][n_nodes] (node positions), and the maps ``node_map`` (new node -> lattice node),
    ``elem_map`` (new element -> lattice element) and ``qp_map`` (new point -> lattice point)."""
    box = d["mesh"]
    assert isinstance(box, Mesh)
    rng = _rng(d["cfg"].cfg_id, STREAM_UNSTRUCT)
    P, Q = box.p + 1, box.q
    conn_l = lattice_connectivity(box)
    # element removal: a cylindrical hole along y
    e = np.arange(box.n_elem)
    ex, ez = e % box.nx, e // (box.nx * box.ny)
    cx = (ex + 0.5) * box.lx / box.nx - 0.5 * box.lx
    cz = (ez + 0.5) * box.lz / box.nz - 0.5 * box.lz
    keep = np.nonzero(cx * cx + cz * cz >= hole_radius * hole_radius)[0]
    elem_map = rng.permutation(keep) if shuffle_elements else keep
    ne = len(elem_map)
    rots = cube_rotations()
    rid = rng.integers(0, len(rots), size=ne) if rotate else np.zeros(ne, dtype=np.int64)
    if not rotate:
        rots = [np.eye(3, dtype=np.int64)]
    nidx = np.stack([rotated_local_index(R, P) for R in rots])  # [24][P^3]
    qidx = np.stack([rotated_local_index(R, Q) for R in rots])  # [24][Q^3]
    conn_old = conn_l[elem_map[:, None], nidx[rid]]  # lattice node ids, rotated local order
    used, first = np.unique(conn_old.reshape(-1), return_index=True)
    if node_order == "random":
        node_map = rng.permutation(used)
    elif node_order == "first_touch":
        node_map = used[np.argsort(first, kind="stable")]
    else:
        raise ValueError(node_order)
    new_of_old = np.full(box.n_nodes, -1, dtype=np.int64)
    new_of_old[node_map] = np.arange(len(node_map))
    conn = new_of_old[conn_old].astype(np.int32)
    qp_map = (elem_map[:, None] * Q ** 3 + qidx[rid]).reshape(-1)
    mesh = UMesh(box.p, ne, len(node_map), box)
    if d.get("X") is not None:
        X = d["X"][:, node_map]
    else:
        gll = gll_points(box.p)
        xs = _coords_1d(box.nx, box.p, box.lx, gll)
        ys = _coords_1d(box.ny, box.p, box.ly, gll)
        zs = _coords_1d(box.nz, box.p, box.lz, gll)
        nx1, ny1, _ = box.node_dims
        X = np.stack([xs[node_map % nx1], ys[(node_map // nx1) % ny1], zs[node_map // (nx1 * ny1)]])
    out = dict(d, mesh=mesh, conn=conn, X=np.ascontiguousarray(X), node_map=node_map, elem_map=elem_map,
               qp_map=qp_map, hole_radius=hole_radius)
    for k in ("z", "dz", "v_rand", "v_top"):
        if k in d:
            out[k] = np.ascontiguousarray(d[k][:, node_map])
    for k in ("dz", "v_rand"):
        if k in out:
            out[k] /= np.linalg.norm(out[k])
    out["phi_n"] = np.ascontiguousarray(d["phi_n"][node_map])
    out["state"] = np.ascontiguousarray(d["state"][:, qp_map])
    out["phase"] = np.ascontiguousarray(d["phase"][qp_map])
    if "xstate" in d:
        out["xstate"] = np.ascontiguousarray(d["xstate"][:, qp_map])
    out["vol_frac"] = float(out["phase"].mean())
    return out
