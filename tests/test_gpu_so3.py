"""GPU parity of SO(3) plans (Plan(..., group="so3")) against the CPU SO(3)
oracle: forward, inverse and adjoint in full at small bandlimits, sampled
coefficients and sample points at larger ones, the adjoint identity and an
exact round trip at B = 64 (integer degrees, N = 2B periodic nodes per angle,
gamma over [-pi, pi))."""
import numpy as np
import pytest
import torch

import paper_2605_23923_amd as su2
import synth
from _errlog import record
from oracle import so3 as oso3

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-10, "c64": 1e-6, "c64_bf16x3": 1e-5}
WORST = 10  # the worst element may be this many times the normwise bound
CDT = {"c128": np.complex128, "c64": np.complex64, "c64_bf16x3": np.complex64}


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    return t.detach().cpu().numpy()


def _check(got, ref, tol, what):
    got = np.asarray(got).astype(np.complex128).reshape(-1)
    ref = np.asarray(ref).astype(np.complex128).reshape(-1)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    worst = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"{what}: rel {rel:.3e} worst {worst:.3e}", flush=True)
    record(what, rel, worst, tol=tol)
    assert rel <= tol and worst <= WORST * tol, f"{what}: rel {rel:.3e} worst {worst:.3e} tol {tol}"


def test_so3_layout_and_shapes():
    for B in (8, 16, 32, 64):
        plan = su2.Plan(B, 2, "c64", group="so3")
        assert plan.ncoef == oso3.num_coeffs(B) == synth.num_coeffs_so3(B)
        assert plan.sample_shape == (2, 2 * B, 2 * B, 2 * B)


@pytest.mark.parametrize("dtype", ["c128", "c64", "c64_bf16x3"])
@pytest.mark.parametrize("B", [4, 8, 12, 16])
def test_so3_matches_oracle(B, dtype):
    """B = 8, 16: register-resident rings; B = 4, 12 (N = 8, 24): the generic
    rings."""
    batch = 2
    plan = su2.Plan(B, batch, dtype, group="so3")
    x = synth.samples_uniform(B, batch, seed=2100 + B, dtype=CDT[dtype])
    _check(_host(plan.forward(_dev(x))), np.stack([oso3.forward(B, v) for v in x]), TOL[dtype],
           f"so3 forward B={B} {dtype}")
    c = synth.coeffs_so3(B, batch, seed=2200 + B, dtype=CDT[dtype])
    _check(_host(plan.inverse(_dev(c))), np.stack([oso3.inverse(B, v) for v in c]), TOL[dtype],
           f"so3 inverse B={B} {dtype}")
    _check(_host(plan.adjoint(_dev(c))), np.stack([oso3.adjoint(B, v) for v in c]), TOL[dtype],
           f"so3 adjoint B={B} {dtype}")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("B,batch", [(32, 3), (64, 8)])
def test_so3_sampled_against_oracle(B, batch, dtype):
    """Larger bandlimits: sampled coefficients of the forward, sampled points
    of the inverse (a ragged batch, the last signal checked)."""
    plan = su2.Plan(B, batch, dtype, group="so3")
    rng = np.random.default_rng(B + 7)
    x = synth.samples_uniform(B, batch, seed=2300 + B, dtype=CDT[dtype])
    sel = rng.choice(oso3.num_coeffs(B), 24, replace=False)
    sel[0] = 0                                          # l = 0
    sel[1] = oso3.num_coeffs(B) - 1                     # l = L-1, m = n = L-1
    got = _host(plan.forward(_dev(x)))[batch - 1][sel]
    _check(got, oso3.forward(B, x[batch - 1], sel), TOL[dtype], f"so3 forward B={B} {dtype} sampled")
    if B <= 32:
        c = synth.coeffs_so3(B, batch, seed=2400 + B, spectrum="decay", dtype=CDT[dtype])
        N = 2 * B
        pts = rng.choice(N ** 3, 24, replace=False)
        got = _host(plan.inverse(_dev(c))).reshape(batch, -1)[batch - 1][pts]
        _check(got, oso3.inverse_at(B, c[batch - 1], pts), TOL[dtype], f"so3 inverse B={B} {dtype} sampled")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_so3_adjoint_identity_b64(dtype):
    """<forward x, c> = <x, adjoint c> on the whole batch."""
    B, batch = 64, 4
    plan = su2.Plan(B, batch, dtype, group="so3")
    x = synth.samples_uniform(B, batch, seed=2500, dtype=CDT[dtype])
    c = synth.coeffs_so3(B, batch, seed=2501, dtype=CDT[dtype])
    fx = _host(plan.forward(_dev(x))).astype(np.complex128)
    ac = _host(plan.adjoint(_dev(c))).astype(np.complex128)
    lhs = np.vdot(fx, c.astype(np.complex128))
    rhs = np.vdot(x.astype(np.complex128), ac)
    scale = np.linalg.norm(fx) * np.linalg.norm(c)
    print(f"so3 adjoint identity {dtype}: {abs(lhs - rhs) / scale:.3e}", flush=True)
    assert abs(lhs - rhs) <= (1e-12 if dtype == "c128" else 1e-5) * scale


@pytest.mark.parametrize("dtype", ["c128", "c64", "c64_bf16x3"])
def test_so3_generic_rings_sampled_b24(dtype):
    """N = 48 (generic rings): sampled coefficients and sample points."""
    B, batch = 24, 3
    plan = su2.Plan(B, batch, dtype, group="so3")
    rng = np.random.default_rng(29)
    x = synth.samples_uniform(B, batch, seed=2800, dtype=CDT[dtype])
    sel = rng.choice(oso3.num_coeffs(B), 24, replace=False)
    sel[0] = oso3.num_coeffs(B) - 1
    _check(_host(plan.forward(_dev(x)))[batch - 1][sel], oso3.forward(B, x[batch - 1], sel), TOL[dtype],
           f"so3 forward B={B} {dtype} sampled")
    c = synth.coeffs_so3(B, batch, seed=2801, spectrum="decay", dtype=CDT[dtype])
    pts = rng.choice((2 * B) ** 3, 24, replace=False)
    _check(_host(plan.inverse(_dev(c))).reshape(batch, -1)[batch - 1][pts], oso3.inverse_at(B, c[batch - 1], pts),
           TOL[dtype], f"so3 inverse B={B} {dtype} sampled")


@pytest.mark.parametrize("dtype", ["c128", "c64", "c64_bf16x3"])
def test_so3_b128(dtype):
    """N = 256 rings: sampled forward coefficients against the oracle, the
    adjoint identity, and (FP64) the exact round trip."""
    B, batch = 128, 2
    plan = su2.Plan(B, batch, dtype, group="so3")
    rng = np.random.default_rng(31)
    x = synth.samples_uniform(B, batch, seed=2900, dtype=CDT[dtype])
    fx = _host(plan.forward(_dev(x)))
    sel = rng.choice(oso3.num_coeffs(B), 8, replace=False)
    sel[0] = oso3.num_coeffs(B) - 1
    _check(fx[batch - 1][sel], oso3.forward(B, x[batch - 1], sel), TOL[dtype], f"so3 forward B={B} {dtype} sampled")
    c = synth.coeffs_so3(B, batch, seed=2901, spectrum="decay", dtype=CDT[dtype])
    ac = _host(plan.adjoint(_dev(c))).astype(np.complex128)
    lhs = np.vdot(fx.astype(np.complex128), c.astype(np.complex128))
    rhs = np.vdot(x.astype(np.complex128), ac)
    err = abs(lhs - rhs) / (np.linalg.norm(fx) * np.linalg.norm(c))
    print(f"so3 adjoint identity B=128 {dtype}: {err:.3e}", flush=True)
    assert err <= (1e-12 if dtype == "c128" else 1e-5)
    if dtype == "c128":
        back = _host(plan.forward(plan.inverse(_dev(c))))
        _check(back, c, 1e-11, "so3 round trip B=128")


def test_so3_round_trip_b64():
    """Bandlimited coefficients -> samples -> the same coefficients (exact quadrature)."""
    B, batch = 64, 4
    plan = su2.Plan(B, batch, "c128", group="so3")
    c = synth.coeffs_so3(B, batch, seed=2600, spectrum="decay")
    back = _host(plan.forward(plan.inverse(_dev(c))))
    _check(back, c, 1e-12, "so3 round trip B=64")


def test_so3_autograd_backward_is_adjoint():
    B, batch = 16, 2
    plan = su2.Plan(B, batch, "c128", group="so3")
    x = _dev(synth.samples_uniform(B, batch, seed=2700)).requires_grad_(True)
    g = _dev(synth.coeffs_so3(B, batch, seed=2701))
    f = su2.SU2Transform.apply(x, plan)
    f.backward(g)
    _check(_host(x.grad), np.stack([oso3.adjoint(B, v) for v in _host(g)]), 1e-10, "so3 backward")


def test_so3_plan_options_rejected():
    for kw in (dict(dtype="c64", tables="on_the_fly"), dict(dtype="c64", real=True)):
        with pytest.raises(su2.SU2Error) as ei:
            su2.Plan(8, 1, group="so3", **kw)
        assert ei.value.status == 2
    plan = su2.Plan(8, 1, "c128", group="so3")
    with pytest.raises(su2.SU2Error) as ei:
        plan.beta_forward_shifted(torch.zeros(plan.coeff_shape, dtype=torch.complex128, device="cuda"), depth=1)
    assert ei.value.status == 1
