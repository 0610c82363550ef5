"""FP32 p-multigrid and the Newton step on mapped (curved) elements (Section 4's geometric
factors in every level apply): the linearisation record, the FP32 fine apply and the FP64
apply from the stored linearisation against the oracle, coarse levels as Galerkin products,
the Jacobi diagonals, the V-cycle, and one Newton update against the dense solve of the
oracle's assembled constrained Jacobian.

Bars: 1e-5 (FP32 levels, diagonals), 1e-12 (stored FP64 linearisation); the Newton bars as
on the box.
"""
import numpy as np
import pytest

from paper_2607_21150_amd import inputs as I
from test_gpu_mg import gmres, lin_ctx, prolong_np, restrict_np
from test_gpu_step import assembled_jacobian, constrained_start, uniaxial_faces

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
FP32_TOL = 1e-5
FP64_TOL = 1e-12


@pytest.fixture(scope="module")
def pf():
    from paper_2607_21150_amd import pfmf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pfmf.load()
    return pfmf


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)


RECORD_CASES = [("plastic", 2, 4), ("plastic", 3, 2), ("base", 3, 3), ("compress", 3, 2), ("voce", 2, 3),
                ("plastic", 4, 2), ("ex3", 2, 4), ("ex3", 3, 2), ("ex3", 4, 2)]
# order 4 scatters by element colours only: one scatter mode there
RECORD_SCATTER = [c + (sc,) for c in RECORD_CASES for sc in (("colour",) if c[1] == 4 else ("colour", "brick_buffer"))]


@pytest.mark.parametrize("variant,p,n,scatter", RECORD_SCATTER)
def test_curved_fp32_and_stored_apply(pf, oracle_lib, variant, p, n, scatter):
    print(f"case curved record applies Q{p} {variant} n={n} {scatter}", flush=True)
    d = I.make_inputs("C1", variant, p=p, n=n, geometry="curved")
    ctx = pf.Context.from_inputs(d)
    ctx.set_scatter(scatter)
    ctx.linearize(dev(d["z"]))
    y32 = ctx.apply_jacobian_f32(0, dev(d["dz"], torch.float32)).double().cpu().numpy()
    ylin = ctx.apply_jacobian_lin(dev(d["dz"])).cpu().numpy()
    ctx.check()
    ref = oracle_lib.Oracle.from_inputs(d).jacobian(d["z"], d["dz"])
    assert relerr(y32, ref) <= FP32_TOL, relerr(y32, ref)
    assert relerr(ylin, ref) <= FP64_TOL, relerr(ylin, ref)


@pytest.mark.parametrize("p,level,variant", [(2, 1, "plastic"), (3, 1, "plastic"), (3, 2, "plastic"),
                                             (4, 1, "plastic"), (4, 2, "plastic"), (4, 3, "plastic"),
                                             (3, 2, "ex3"), (4, 1, "ex3")])
def test_curved_coarse_operator_is_galerkin_product(pf, oracle_lib, p, level, variant):
    """A_c = P^T A_f P on the curved mesh (the order-1 level, the last of each list, assembled
    from element matrices); ex3: with branches in parallel."""
    d = I.make_inputs("C1", variant, p=p, n=2, geometry="curved")
    ctx = lin_ctx(pf, d)
    m = d["mesh"]
    orc = oracle_lib.Oracle.from_inputs(d)
    rng = np.random.default_rng(1)
    _, nl = ctx.level_info(level)
    xc = rng.standard_normal((4, nl))
    yc = ctx.apply_jacobian_f32(level, dev(xc, torch.float32)).cpu().numpy()
    Pxc = xc
    for q in range(m.p - level, m.p):
        Pxc, _ = prolong_np(Pxc, m.nx, q + 1, q)
    ref = orc.jacobian(d["z"], Pxc)
    for q in range(m.p, m.p - level, -1):
        ref = restrict_np(ref, m.nx, q, q - 1)
    assert relerr(yc, ref) <= FP32_TOL, relerr(yc, ref)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_curved_fine_diagonal_matches_oracle_element_matrices(pf, oracle_lib, p):
    d = I.make_inputs("C1", "plastic", p=p, n=2, geometry="curved")
    ctx = lin_ctx(pf, d)
    diag = ctx.level_diagonal(0).cpu().numpy()
    orc = oracle_lib.Oracle.from_inputs(d)
    m = d["mesh"]
    ref = np.zeros((4, m.n_nodes))
    nP = (m.p + 1) ** 3
    for e in range(m.n_elem):
        K = orc.element_jacobian(d["z"], e)
        nodes = orc.element_nodes(e)
        dk = np.diag(K).reshape(4, nP)
        for f in range(4):
            np.add.at(ref[f], nodes, dk[f])
    assert relerr(diag, ref) <= FP32_TOL, relerr(diag, ref)


@pytest.mark.parametrize("p,level", [(3, 1), (2, 1)])
def test_curved_coarse_diagonal_matches_unit_applies(pf, p, level):
    """The diagonal of a coarse level (generic level kernel on order 3 -> 2, element-matrix
    stencil on order 2 -> 1) equals the level apply on unit vectors."""
    d = I.make_inputs("C1", "plastic", p=p, n=2, geometry="curved")
    ctx = lin_ctx(pf, d)
    _, n1 = ctx.level_info(level)
    diag = ctx.level_diagonal(level).cpu().numpy()
    ref = np.zeros((4, n1))
    e = torch.zeros((4, n1), dtype=torch.float32, device="cuda")
    for f in range(4):
        for i in range(n1):
            e.zero_()
            e[f, i] = 1.0
            ref[f, i] = float(ctx.apply_jacobian_f32(level, e)[f, i])
    assert relerr(diag, ref) <= FP32_TOL, relerr(diag, ref)


def test_curved_vcycle_preconditioned_gmres(pf):
    d = I.make_inputs("C1", "base", p=3, n=4, geometry="curved")
    ctx = lin_ctx(pf, d)
    rng = np.random.default_rng(3)
    A = lambda v: ctx.apply_jacobian_f32(0, v)
    b = A(dev(rng.standard_normal((4, d["mesh"].n_nodes)), torch.float32))
    h_prec = gmres(A, b, prec=lambda v: ctx.pmg_vcycle(v), tol=1e-5, maxit=60)
    h_none = gmres(A, b, prec=None, tol=1e-5, maxit=60)
    print("curved GMRES its with V-cycle", len(h_prec) - 1, h_prec[-1], "without", len(h_none) - 1, h_none[-1],
          flush=True)
    assert h_prec[-1] < 1e-5
    assert len(h_prec) < len(h_none) or h_none[-1] > 1e-5


@pytest.mark.parametrize("variant", ["base", "plastic", "ex3"])
def test_curved_newton_update_matches_dense_solve(pf, oracle_lib, variant):
    """One Newton update on the curved mesh (planar boundary faces, so the box's uniaxial
    faces apply): FGMRES with the V-cycle reaches 1e-11 and the update agrees with the dense
    solve of the oracle's assembled constrained Jacobian."""
    print(f"case curved newton update C1 {variant}", flush=True)
    d = I.make_inputs("C1", variant, geometry="curved")
    z0, M = constrained_start(d)
    orc = oracle_lib.Oracle.from_inputs(d)
    ctx = pf.Context.from_inputs(d)
    ctx.set_dirichlet(uniaxial_faces())
    z = dev(z0)
    rep = ctx.newton_step(z, rtol=1e-11, restart=40, max_iters=400)
    print(rep, flush=True)
    assert rep["converged"] == 1
    dz = (z.cpu().numpy() - z0).reshape(-1)
    free = ~M.reshape(-1)
    assert np.all(dz[~free] == 0.0)
    r = orc.residual(z0).reshape(-1)
    K = assembled_jacobian(orc, d["mesh"], z0)
    Kff = K[np.ix_(free, free)]
    ref = np.linalg.solve(Kff, -r[free])
    kappa = np.linalg.cond(Kff)
    err = np.linalg.norm(dz[free] - ref) / np.linalg.norm(ref)
    res = np.linalg.norm(Kff @ dz[free] + r[free]) / np.linalg.norm(r[free])
    print("kappa", kappa, "rel err", err, "system residual", res, flush=True)
    assert res <= 1e-9
    assert err <= max(10 * kappa * 1e-11, 1e-9)


def test_curved_newton_converges_on_small_mesh(pf):
    """Newton iterations on the curved mesh under the base loading: the constrained residual
    falls by 1e-8 in five updates, as on the box."""
    d = I.make_inputs("C1", "base", geometry="curved")
    z0, M = constrained_start(d)
    ctx = pf.Context.from_inputs(d)
    ctx.set_dirichlet(uniaxial_faces())
    z = dev(z0)
    Mt = torch.as_tensor(M).cuda()
    hist = []
    for k in range(6):
        r = ctx.apply_residual(z)
        r[Mt] = 0
        hist.append(float(torch.linalg.norm(r)))
        if k < 5:
            ctx.newton_step(z, rtol=1e-10, restart=40, max_iters=400)
    print("curved Newton residual history", hist, flush=True)
    assert hist[-1] <= 1e-8 * hist[0]
    assert hist[-1] < 0.1 * hist[-2]
