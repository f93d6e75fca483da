"""GPU parity of plans whose Wigner-d values are generated inside the beta
contraction kernels (tables="on_the_fly"), against the CPU oracle and against
the stored-table plans.

Tolerances as in test_gpu_parity.py (1e-10 FP64, 1e-6 FP32; the recurrence
runs in FP64 either way).  Stored and generated tables come from the same
FP64 recurrence with coefficients rounded differently (device FP64 vs host
long double), so the two plans agree to rounding of the table values."""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_23923_amd as su2
import synth
from _errlog import record

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-10, "c64": 1e-6}
WORST = 10  # the worst element may be this many times the normwise bound
NPDT = {"c128": np.complex128, "c64": np.complex64}


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def _check(got, ref, tol, what):
    got = np.asarray(got, dtype=np.complex128).reshape(-1)
    ref = np.asarray(ref, dtype=np.complex128).reshape(-1)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    worst = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"{what}: rel {rel:.3e} worst {worst:.3e}", flush=True)
    record(what, rel, worst, tol=tol)
    assert rel <= tol and worst <= WORST * tol, f"{what}: rel {rel:.3e} worst {worst:.3e} tol {tol}"


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("B", [1, 2, 3, 4, 6, 8, 12, 16])
def test_otf_matches_oracle(B, dtype):
    batch = 3
    plan = su2.Plan(B, batch, dtype, tables="on_the_fly")
    x = synth.samples_uniform(B, batch, seed=700 + B, dtype=NPDT[dtype])
    c = synth.coeffs(B, batch, seed=800 + B, dtype=NPDT[dtype])
    _check(_host(plan.forward(_dev(x))), np.stack([oracle.forward(B, v) for v in x]), TOL[dtype],
           f"otf forward B={B} {dtype}")
    _check(_host(plan.inverse(_dev(c))), np.stack([oracle.inverse(B, v) for v in c]), TOL[dtype],
           f"otf inverse B={B} {dtype}")
    _check(_host(plan.adjoint(_dev(c))), np.stack([oracle.adjoint(B, v) for v in c]), TOL[dtype],
           f"otf adjoint B={B} {dtype}")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("B,batch", [(24, 3), (16, 21), (64, 32)])
def test_otf_equals_stored_tables(B, batch, dtype):
    x = synth.samples_uniform(B, batch, seed=910, dtype=NPDT[dtype])
    c = synth.coeffs(B, batch, seed=911, spectrum="decay", dtype=NPDT[dtype])
    po = su2.Plan(B, batch, dtype, tables="on_the_fly")
    ps = su2.Plan(B, batch, dtype)
    tol = 1e-13 if dtype == "c128" else 1e-6
    _check(_host(po.forward(_dev(x))), _host(ps.forward(_dev(x))), tol, f"otf vs stored forward B={B} {dtype}")
    _check(_host(po.inverse(_dev(c))), _host(ps.inverse(_dev(c))), tol, f"otf vs stored inverse B={B} {dtype}")
    _check(_host(po.adjoint(_dev(c))), _host(ps.adjoint(_dev(c))), tol, f"otf vs stored adjoint B={B} {dtype}")
    # sampled against the oracle as well
    rng = np.random.default_rng(B)
    sel = rng.choice(oracle.num_coeffs(B), 64, replace=False)
    _check(_host(po.forward(_dev(x)))[1][sel], oracle.forward(B, x[1], sel), TOL[dtype],
           f"otf forward B={B} {dtype} sampled")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_otf_b128_round_trip_and_samples(dtype):
    """B = 128 with generated tables (the stored FP64 table would be 1.45 GB)."""
    B, batch = 128, 2
    plan = su2.Plan(B, batch, dtype, tables="on_the_fly")
    c = synth.coeffs(B, batch, seed=4, dtype=NPDT[dtype])
    x = plan.inverse(_dev(c))
    _check(_host(plan.forward(x)), c, 1e-11 if dtype == "c128" else 2e-6, f"otf round trip B=128 {dtype}")
    rng = np.random.default_rng(5)
    pts = rng.choice((2 * B) ** 3, 16, replace=False)
    xs = _host(x)
    del x
    _check(xs[0].reshape(-1)[pts], oracle.inverse(B, c[0], pts), TOL[dtype], f"otf inverse B=128 {dtype}")


def test_otf_plan_holds_no_table():
    B, batch = 64, 1
    po = su2.Plan(B, batch, "c128", tables="on_the_fly")
    ps = su2.Plan(B, batch, "c128")
    table = su2.num_coeffs(B) * 2 * B * 8
    assert ps.device_bytes() - po.device_bytes() > 0.9 * table
    with pytest.raises(su2.SU2Error) as ei:
        po.dtable(0, 0)
    assert ei.value.status == 2
    with pytest.raises(su2.SU2Error):
        su2.Plan(8, 1, "c64_bf16x3", tables="on_the_fly")
