"""GPU parity of real-signal plans (Plan(..., real=True)) against the CPU
oracle: forward of real samples (all coefficients, half computed and half by
the Hermitian relation), inverse and adjoint as the real part of the complex
results, equality with complex plans on the same data, exact round trip, and
the autograd backward (real adjoint) against central differences."""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_23923_amd as su2
import synth
from _errlog import record

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-10, "c64": 1e-6, "c64_bf16x3": 1e-5}
WORST = 10  # the worst element may be this many times the normwise bound
RDT = {"c128": np.float64, "c64": np.float32, "c64_bf16x3": np.float32}
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


def _real_samples(B, batch, seed, dtype):
    return synth.samples_uniform(B, batch, seed=seed).real.astype(RDT[dtype])


@pytest.mark.parametrize("dtype", ["c128", "c64", "c64_bf16x3"])
@pytest.mark.parametrize("B", [4, 8, 12, 16])
def test_real_plan_matches_oracle(B, dtype):
    """B = 8, 16: the half-spectrum rings; B = 4, 12 (N = 8, 24): the generic
    rings with real samples in and the real part out."""
    batch = 3
    plan = su2.Plan(B, batch, dtype, real=True)
    x = _real_samples(B, batch, 1200 + B, dtype)
    _check(_host(plan.forward(_dev(x))), np.stack([oracle.forward(B, v.astype(np.complex128)) for v in x]),
           TOL[dtype], f"real forward B={B} {dtype}")
    c = synth.coeffs(B, batch, seed=1300 + B, dtype=CDT[dtype])   # not Hermitian: the real part is returned
    gi = _host(plan.inverse(_dev(c)))
    ga = _host(plan.adjoint(_dev(c)))
    assert gi.dtype == RDT[dtype] and ga.dtype == RDT[dtype]
    _check(gi, np.stack([oracle.inverse(B, v).real for v in c]), TOL[dtype], f"real inverse B={B} {dtype}")
    _check(ga, np.stack([oracle.adjoint(B, v).real for v in c]), TOL[dtype], f"real adjoint B={B} {dtype}")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("B,batch", [(32, 5), (64, 32)])
def test_real_plan_equals_complex_plan(B, batch, dtype):
    x = _real_samples(B, batch, 1400 + B, dtype)
    c = synth.coeffs(B, batch, seed=1500 + B, spectrum="decay", dtype=CDT[dtype])
    pr = su2.Plan(B, batch, dtype, real=True)
    pc = su2.Plan(B, batch, dtype)
    tol = 1e-13 if dtype == "c128" else 2e-6
    _check(_host(pr.forward(_dev(x))), _host(pc.forward(_dev(x.astype(CDT[dtype])))), tol,
           f"real vs complex forward B={B} {dtype}")
    _check(_host(pr.inverse(_dev(c))), _host(pc.inverse(_dev(c))).real, tol, f"real vs complex inverse B={B} {dtype}")
    _check(_host(pr.adjoint(_dev(c))), _host(pc.adjoint(_dev(c))).real, tol, f"real vs complex adjoint B={B} {dtype}")
    rng = np.random.default_rng(B)
    sel = rng.choice(oracle.num_coeffs(B), 40, replace=False)
    _check(_host(pr.forward(_dev(x)))[batch - 1][sel], oracle.forward(B, x[batch - 1].astype(np.complex128), sel),
           TOL[dtype], f"real forward B={B} {dtype} sampled")


@pytest.mark.parametrize("dtype", ["c128", "c64", "c64_bf16x3"])
@pytest.mark.parametrize("B,batch", [(24, 3), (128, 2)])
def test_real_io_plans_bitwise_equal_complex_plans(B, batch, dtype):
    """Bandlimits without the half-spectrum rings (N = 48 generic, N = 256):
    the complex kernels run on the real samples, so forward equals a complex
    plan's on the same samples, and inverse and adjoint equal the real part of
    a complex plan's, bit for bit; sampled coefficients and points against the
    oracle."""
    x = _real_samples(B, batch, 1800 + B, dtype)
    c = synth.coeffs(B, batch, seed=1900 + B, spectrum="decay", dtype=CDT[dtype])
    pr = su2.Plan(B, batch, dtype, real=True)
    fr = _host(pr.forward(_dev(x)))
    ir = _host(pr.inverse(_dev(c)))
    ar = _host(pr.adjoint(_dev(c)))
    pr.close()
    pc = su2.Plan(B, batch, dtype)
    fc = _host(pc.forward(_dev(x.astype(CDT[dtype]))))
    assert np.array_equal(fr, fc), "forward"
    assert np.array_equal(ir, _host(pc.inverse(_dev(c))).real), "inverse"
    assert np.array_equal(ar, _host(pc.adjoint(_dev(c))).real), "adjoint"
    pc.close()
    rng = np.random.default_rng(B)
    sel = rng.choice(oracle.num_coeffs(B), 24, replace=False)
    sel[0] = oracle.num_coeffs(B) - 1
    _check(fr[batch - 1][sel], oracle.forward(B, x[batch - 1].astype(np.complex128), sel), TOL[dtype],
           f"real forward B={B} {dtype} sampled")
    N = 2 * B
    pts = rng.choice(N ** 3, 24, replace=False)
    _check(ir.reshape(batch, -1)[batch - 1][pts], oracle.inverse(B, c[batch - 1], pts).real, TOL[dtype],
           f"real inverse B={B} {dtype} sampled")


@pytest.mark.parametrize("B,batch", [(16, 3), (64, 32)])
def test_real_plan_split_bf16_equals_complex_plan(B, batch):
    """Half-spectrum rings with the split-BF16 contraction: the same values as a
    split-BF16 complex plan on the same samples, to the mode's rounding."""
    x = _real_samples(B, batch, 2000 + B, "c64_bf16x3")
    c = synth.coeffs(B, batch, seed=2050 + B, spectrum="decay", dtype=np.complex64)
    pr = su2.Plan(B, batch, "c64_bf16x3", real=True)
    pc = su2.Plan(B, batch, "c64_bf16x3")
    _check(_host(pr.forward(_dev(x))), _host(pc.forward(_dev(x.astype(np.complex64)))), TOL["c64_bf16x3"],
           f"real vs complex forward B={B} c64_bf16x3")
    _check(_host(pr.inverse(_dev(c))), _host(pc.inverse(_dev(c))).real, TOL["c64_bf16x3"],
           f"real vs complex inverse B={B} c64_bf16x3")
    _check(_host(pr.adjoint(_dev(c))), _host(pc.adjoint(_dev(c))).real, TOL["c64_bf16x3"],
           f"real vs complex adjoint B={B} c64_bf16x3")


def test_real_round_trip_b64():
    """Hermitian bandlimited coefficients -> real samples -> the same coefficients."""
    B, batch = 64, 4
    pc = su2.Plan(B, batch, "c128")
    pr = su2.Plan(B, batch, "c128", real=True)
    c = synth.coeffs(B, batch, seed=1600, spectrum="decay")
    x = pc.inverse(_dev(c))
    x_real = x.real.contiguous()
    herm = _host(pc.forward(x_real.to(torch.complex128)))   # coefficients of the real part (Hermitian)
    xr = pr.inverse(_dev(herm))           # real samples
    _check(_host(xr), _host(x_real), 1e-12, "real inverse of Hermitian coefficients B=64")
    back = _host(pr.forward(xr))
    _check(back, herm, 1e-12, "real round trip B=64")


def test_real_autograd_matches_central_differences():
    B, batch = 8, 1
    plan = su2.Plan(B, batch, "c128", real=True)
    x0 = _real_samples(B, batch, 1700, "c128")
    T = synth.coeffs(B, batch, seed=1701)
    w = np.concatenate([np.full((tl + 1) ** 2, tl + 1.0) for tl in range(B)])
    Tt, wt = _dev(T), _dev(w)

    def loss(xt):
        f = su2.SU2Transform.apply(xt, plan)
        return (wt * (f - Tt).abs() ** 2).sum()

    x = _dev(x0).requires_grad_(True)
    loss(x).backward()
    g = x.grad.detach().cpu().numpy().reshape(-1)
    rng = np.random.default_rng(5)
    h = 1e-3
    for _ in range(6):
        v = rng.standard_normal(x0.size)
        v /= np.linalg.norm(v)
        vt = _dev(v.reshape(x0.shape))
        with torch.no_grad():
            fd = (loss(_dev(x0) + h * vt) - loss(_dev(x0) - h * vt)).item() / (2 * h)
        an = float(np.dot(g, v))
        assert abs(fd - an) <= 1e-8 * max(1.0, abs(fd)), (fd, an)


def test_real_plan_options_rejected():
    for kw in (dict(dtype="c64", tables="on_the_fly"), dict(dtype="c64", group="so3")):
        with pytest.raises(su2.SU2Error) as ei:
            su2.Plan(8, 1, real=True, **kw)
        assert ei.value.status == 2
    plan = su2.Plan(8, 1, "c64", real=True)
    with pytest.raises(TypeError):
        plan.forward(torch.zeros((1, 16, 16, 16), dtype=torch.complex64, device="cuda"))
