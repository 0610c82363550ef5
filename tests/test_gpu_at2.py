"""HIP library with the AT2 crack regularisation (eq:AT1-AT2: alpha = phi^2, c0 = 2) against
the oracle: FP64 residual, Jacobian, adjoint with parameter partials, the FP64 Jacobian from
the stored linearisation and the FP32 fine-level apply.

Bars: 1e-12 (FP64), 1e-5 (FP32), relative L2.
"""
import numpy as np
import pytest

from paper_2607_21150_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
FP64_TOL = 1e-12
FP32_TOL = 1e-5


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


@pytest.mark.parametrize("variant,p,n", [("plastic", 2, 4), ("base", 3, 3), ("plastic", 3, 2), ("plastic", 4, 2),
                                         ("compress", 4, 2), ("voce", 3, 2)])
def test_at2_fp64_fp32(pf, oracle_lib, variant, p, n):
    print(f"case AT2 {variant} p={p} n={n}", flush=True)
    d = I.make_inputs("C1", variant, p=p, n=n, at=2)
    assert d["fracture"].at == 2
    orc = oracle_lib.Oracle.from_inputs(d)
    ctx = pf.Context.from_inputs(d)
    z, dz, v = dev(d["z"]), dev(d["dz"]), dev(d["v_rand"])
    r = ctx.apply_residual(z).cpu().numpy()
    y = ctx.apply_jacobian(z, dz).cpu().numpy()
    gz, gp = ctx.apply_adjoint(z, v)
    ctx.linearize(z)
    ylin = ctx.apply_jacobian_lin(dz).cpu().numpy()
    y32 = ctx.apply_jacobian_f32(0, dev(d["dz"], torch.float32)).double().cpu().numpy()
    ctx.check()
    yref = orc.jacobian(d["z"], d["dz"])
    assert relerr(r, orc.residual(d["z"])) <= FP64_TOL
    assert relerr(y, yref) <= FP64_TOL
    assert relerr(ylin, yref) <= FP64_TOL
    assert relerr(y32, yref) <= FP32_TOL, relerr(y32, yref)
    gref, gpref = orc.adjoint(d["z"], d["v_rand"])
    assert relerr(gz.cpu().numpy(), gref) <= FP64_TOL
    gp = gp.cpu().numpy()
    for k in range(3):
        scale = max(np.abs(gpref[:, k]).max(), 1e-300)
        assert np.abs(gp[:, k] - gpref[:, k]).max() <= 1e-11 * scale, (k, gp[:, k], gpref[:, k])


@pytest.mark.parametrize("p,n", [(2, 3), (3, 2), (4, 2)])
def test_at2_with_branches(pf, oracle_lib, p, n):
    """AT2 with the third example's branches in parallel (FP64 applies)."""
    print(f"case AT2 ex3 p={p} n={n}", flush=True)
    d = I.make_inputs("C1", "ex3", p=p, n=n, at=2)
    orc = oracle_lib.Oracle.from_inputs(d)
    ctx = pf.Context.from_inputs(d)
    z, dz, v = dev(d["z"]), dev(d["dz"]), dev(d["v_rand"])
    r = ctx.apply_residual(z).cpu().numpy()
    y = ctx.apply_jacobian(z, dz).cpu().numpy()
    gz, gp = ctx.apply_adjoint(z, v)
    ctx.check()
    assert relerr(r, orc.residual(d["z"])) <= FP64_TOL
    assert relerr(y, orc.jacobian(d["z"], d["dz"])) <= FP64_TOL
    gref, gpref = orc.adjoint(d["z"], d["v_rand"])
    assert relerr(gz.cpu().numpy(), gref) <= FP64_TOL
    gp = gp.cpu().numpy()
    for k in range(3):
        scale = max(np.abs(gpref[:, k]).max(), 1e-300)
        assert np.abs(gp[:, k] - gpref[:, k]).max() <= 1e-11 * scale, (k, gp[:, k], gpref[:, k])
