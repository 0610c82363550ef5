"""Adjoint on the GPU: the torch.autograd.Function wrapper, the oracle's gradient and
central finite differences, on the full adjoint workload (Q2, 32^3 elements, 1.1 M DoFs).

Pins (adjoint of the matrix-free residual, Section 4):
* z-gradient and per-phase (Gc, sigma0, visc) gradient equal the oracle's (dense element
  Jacobians transposed) to 1e-12 / 1e-11;
* the reaction loss (top-face u_z rows) has an identically zero Gc-gradient (Gc enters the
  phase-field rows only), and zero sigma0 / visc gradients when no point yields;
* central differences with relative step h = 1e-6 agree with the gradient to 1e-6 (reaction
  loss on the full workload; random cotangent on a small mesh).
"""
import numpy as np
import pytest

from paper_2607_21150_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pf():
    from paper_2607_21150_amd import pfmf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pfmf.load()
    return pfmf


def dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)


def params_of(d):
    return torch.tensor([[p.Gc, p.sigma0, p.visc] for p in d["phases"]], dtype=torch.float64)


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def c4_plastic(pf):
    print("case C4 plastic (full size)", flush=True)
    d = I.make_inputs("C4", "plastic")
    return d, pf.Context.from_inputs(d)


@pytest.mark.parametrize("cot", ["v_top", "v_rand"])
def test_autograd_gradient_matches_oracle(pf, oracle_lib, c4_plastic, cot):
    d, op = c4_plastic
    print(f"autograd vs oracle, cotangent {cot}", flush=True)
    z = dev(d["z"]).requires_grad_(True)
    params = params_of(d).requires_grad_(True)
    v = dev(d[cot])
    r = pf.phase_field_residual(z, params, op)
    loss = torch.sum(r * v)
    loss.backward()
    op.check()
    orc = oracle_lib.Oracle.from_inputs(d)
    gref, gpref = orc.adjoint(d["z"], d[cot])
    gz = z.grad.cpu().numpy()
    assert relerr(gz, gref) <= 1e-12, relerr(gz, gref)
    gp = params.grad.numpy()
    scale = np.abs(gpref).max()
    assert scale > 0
    assert np.abs(gp - gpref).max() <= 1e-11 * scale, (gp, gpref)
    if cot == "v_top":
        assert np.all(gp[:, 0] == 0.0)  # reaction loss: no Gc dependence
        assert np.abs(gp[0, 1]) > 0 and np.abs(gp[0, 2]) > 0  # the matrix yields in this variant


def test_reaction_loss_parameter_gradient_zero_when_elastic(pf):
    print("case C4 base (full size): no point yields", flush=True)
    d = I.make_inputs("C4", "base")
    op = pf.Context.from_inputs(d)
    z = dev(d["z"])
    params = params_of(d).requires_grad_(True)
    r = pf.phase_field_residual(z, params, op)
    torch.sum(r * dev(d["v_top"])).backward()
    assert np.all(params.grad.numpy() == 0.0), params.grad


def smooth_direction(mesh):
    """[4][n_nodes] device field sin(2 pi (k.x) + phase) with a different wavevector per field."""
    P = mesh.p
    X = I._coords_1d(mesh.nx, P, mesh.lx, I.gll_points(P))
    Y = I._coords_1d(mesh.ny, P, mesh.ly, I.gll_points(P))
    Z = I._coords_1d(mesh.nz, P, mesh.lz, I.gll_points(P))
    out = np.empty((4, len(Z), len(Y), len(X)))
    for f, (kx, ky, kz, ph) in enumerate([(1, 2, 1, 0.3), (2, 1, 1, 1.1), (1, 1, 2, 2.0), (1, 1, 1, 0.7)]):
        out[f] = np.sin(2 * np.pi * (kx * X[None, None, :] + ky * Y[None, :, None] + kz * Z[:, None, None]) + ph)
    return dev(out.reshape(4, -1))


def _loss(pf, op, z, params, v):
    with torch.no_grad():
        r = pf.phase_field_residual(z, params, op)
        return float(torch.sum(r * v))


@pytest.mark.parametrize("case,cot", [("C4", "v_top"), ("small", "v_rand"), ("small_voce", "v_rand")])
def test_central_differences(pf, c4_plastic, case, cot):
    """Central differences of L = <v, R(z; params)> with relative step 1e-6 against the adjoint.

    The reaction loss runs on the full adjoint workload. A random cotangent weights every node
    with a random sign, so <v, J w> is a sum with heavy cancellation (about 1/sqrt(n) of its
    terms' size) and a single point whose yield, split or history switch the step crosses
    moves it by ~1e-4: that check runs on a small mesh (Q2, 6^3 elements), where no switch
    lies within the step.
    """
    if case == "C4":
        d, op = c4_plastic
    else:
        d = I.make_inputs("C1", "voce" if case == "small_voce" else "plastic", p=2, n=6)
        op = pf.Context.from_inputs(d)
    print(f"finite differences, {case}, cotangent {cot}", flush=True)
    h = 1e-6
    z0 = dev(d["z"])
    p0 = params_of(d)
    v = dev(d[cot])
    z = z0.clone().requires_grad_(True)
    params = p0.clone().requires_grad_(True)
    torch.sum(pf.phase_field_residual(z, params, op) * v).backward()
    gz, gp = z.grad, params.grad.numpy()

    # z-directions: smooth fields (the solution itself, and a sine mode per field scaled by the
    # field's RMS), so that h is a relative step and the strain change stays ~h relative: the
    # yield, split and history switches are then crossed at almost no point
    rms = torch.sqrt(torch.mean(z0 ** 2, dim=1, keepdim=True))
    for name, w in (("solution", z0.clone()), ("sines", smooth_direction(d["mesh"]) * rms)):
        fd = (_loss(pf, op, z0 + h * w, p0, v) - _loss(pf, op, z0 - h * w, p0, v)) / (2 * h)
        ad = float(torch.sum(gz * w))
        assert abs(fd - ad) <= 1e-6 * abs(ad), (name, fd, ad, abs(fd - ad) / abs(ad))

    # parameters: relative step on each (phase, parameter) with a nonzero value. The loss moves
    # by only ~1e-10 for a 1e-6 relative change of the overstress viscosity, which is at the
    # rounding level of L; that entry takes a 1e-4 relative step instead. It crosses no switch:
    # d dgamma / d visc vanishes with dgamma at the yield surface, so L is smooth in visc.
    for ph in range(p0.shape[0]):
        for k in range(3):
            val = float(p0[ph, k])
            if val == 0.0:
                continue
            hk = 1e-4 if k == 2 else h
            dp = torch.zeros_like(p0)
            dp[ph, k] = hk * val
            fdk = (_loss(pf, op, z0, p0 + dp, v) - _loss(pf, op, z0, p0 - dp, v)) / (2 * hk * val)
            adk = gp[ph, k]
            if adk == 0.0:
                assert fdk == 0.0, (ph, k, fdk)
            else:
                assert abs(fdk - adk) <= 1e-6 * abs(adk), (ph, k, fdk, adk)
    op.set_params(p0.numpy())


def test_gradcheck_small(pf):
    """torch.autograd.gradcheck (fast mode) of the wrapper on the small Q2 case."""
    d = I.make_inputs("C1", "base")
    op = pf.Context.from_inputs(d)
    z = dev(d["z"]).requires_grad_(True)
    p0 = params_of(d)
    # the matrix row only: the particle phase has sigma0 = visc = 0, which a step would make negative
    pm = p0[:1].clone().requires_grad_(True)
    rest = p0[1:]
    assert torch.autograd.gradcheck(lambda zz, mm: pf.phase_field_residual(zz, torch.cat([mm, rest]), op),
                                    (z, pm), eps=1e-7, atol=1e-6, rtol=1e-5, fast_mode=True)
