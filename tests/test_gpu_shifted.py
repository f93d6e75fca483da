"""GPU parity of the forward contraction in the shifted-recurrence
(divide-and-conquer) form of Section 4 against the CPU oracles: the direct
sum (what the transform is), the oracle's own k = 1 / k = 2 projections of
oracle/shifted.py applied to the same ring spectra, and the table contraction
of the same plan.

Tolerance: the form is evaluated in FP64; its shifted polynomials grow where
d is small, so the agreement with the table form is a few 1e-13 relative
rather than 1e-15; FP32 plans are bounded by their FP32 ring spectra (2e-5)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_23923_amd as su2
import synth

pytestmark = pytest.mark.gpu

NPDT = {"c128": np.complex128, "c64": np.complex64}
TOL = {"c128": 1e-10, "c64": 2e-5}


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def _rel(a, r):
    a, r = np.asarray(a).reshape(-1), np.asarray(r).reshape(-1)
    return np.linalg.norm(a - r) / np.linalg.norm(r)


def _shifted(plan, x, depth, block):
    plan.run_stage("ring_forward", x, None)
    return plan.beta_forward_shifted(depth=depth, block=block)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("B", [1, 2, 3, 4, 8, 12, 16])
@pytest.mark.parametrize("depth,block", [(1, 4), (2, 2), (2, 4), (2, 8), (2, 16)])
def test_shifted_forward_matches_oracle(B, dtype, depth, block):
    batch = 3
    x = synth.samples_uniform(B, batch, seed=1000 + B, dtype=NPDT[dtype])
    plan = su2.Plan(B, batch, dtype)
    got = _host(_shifted(plan, _dev(x), depth, block))
    ref = np.stack([oracle.forward(B, v) for v in x])
    rel = _rel(got, ref)
    print(f"shifted depth {depth} block {block} B={B} {dtype}: rel {rel:.3e}", flush=True)
    assert rel <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("depth,block", [(1, 4), (2, 4), (2, 8), (2, 16)])
def test_shifted_equals_table_contraction_b64(dtype, depth, block):
    B, batch = 64, 32
    x = synth.samples_uniform(B, batch, seed=1064, dtype=NPDT[dtype])
    plan = su2.Plan(B, batch, dtype)
    table = _host(plan.forward(_dev(x)))
    got = _host(_shifted(plan, _dev(x), depth, block))
    rel = _rel(got, table)
    print(f"shifted vs table B=64 {dtype} depth {depth}: rel {rel:.3e}", flush=True)
    assert rel <= (1e-12 if dtype == "c128" else 1e-6)
    rng = np.random.default_rng(64)
    sel = rng.choice(oracle.num_coeffs(B), 48, replace=False)
    assert _rel(got[5][sel], oracle.forward(B, x[5], sel)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("B,batch", [(24, 37), (36, 5), (48, 3), (64, 1)])
@pytest.mark.parametrize("depth,block", [(1, 4), (2, 16)])
def test_shifted_matrix_core_forms_ragged(dtype, B, batch, depth, block):
    """Depth 1 and depth 2 with block 16 on the matrix cores take 32 signals
    per workgroup: a second, partial signal tile (37), a batch far below one
    tile (5, 3, 1), one and two row tiles of degrees (B = 24: L <= 12;
    B = 36: L up to 18, with the pairs of L = 17 whose second tile is one row,
    fine polynomials A_{-1} = 0 and B_{-1} = 1 alone; B = 48, 64: L up to 24
    and 32)."""
    x = synth.samples_uniform(B, batch, seed=2000 + B, dtype=NPDT[dtype])
    plan = su2.Plan(B, batch, dtype)
    table = _host(plan.forward(_dev(x)))
    got = _host(_shifted(plan, _dev(x), depth, block))
    rel = _rel(got, table)
    print(f"shifted depth {depth} block {block} vs table B={B} batch={batch} {dtype}: rel {rel:.3e}", flush=True)
    assert rel <= (1e-12 if dtype == "c128" else 1e-6)
    rng = np.random.default_rng(B)
    sel = rng.choice(oracle.num_coeffs(B), 32, replace=False)
    last = batch - 1
    assert _rel(got[last][sel], oracle.forward(B, x[last], sel)) <= TOL[dtype]


def test_shifted_matches_oracle_projections_on_gpu_spectra():
    """The oracle's k = 1 and k = 2 projections of oracle/shifted.py, applied to
    one pair's node values, agree with the GPU stage for that pair's degrees."""
    from oracle import shifted as osh
    B, batch = 8, 1
    N = 2 * B
    x = synth.samples_uniform(B, batch, seed=1108)
    plan = su2.Plan(B, batch, "c128")
    got = _host(_shifted(plan, _dev(x), 2, 2))[0]
    ref = oracle.forward(B, x[0])
    _, beta, _, W = oracle.grid(B)
    xs = np.cos(beta)
    # ring spectrum of pair (m, n) = (1/2, 3/2) from the forward definition:
    # S_k = W_k sum_{j,l} f e^{i(n alpha_j + m gamma_l)} i^{n-m}
    a, b_, g, _ = oracle.grid(B)
    tm, tn = 1, 3
    ph = np.exp(1j * (tn / 2 * a[None, :, None] + tm / 2 * g[None, None, :]))
    S = W * (x[0].reshape(N, N, N) * ph).sum(axis=(1, 2)) * (1j ** ((tn - tm) // 2))
    l0 = 3
    dL = np.array([oracle.wigner_d(l0 + 2, tn, tm, bb) for bb in beta])
    dLm1 = np.array([oracle.wigner_d(l0, tn, tm, bb) for bb in beta])
    for i in range(1, (B - 1 - l0) // 2 + 1):
        r = i - 1
        k1 = osh.projection_k1(S, dL, dLm1, l0 + 2, r, tm, tn, xs)
        k2 = osh.projection_k2(S, dL, dLm1, l0 + 2, (r // 2) * 2, r % 2, tm, tn, xs)
        idx = oracle.coeff_index(l0 + 2 * i, tm, tn)
        assert abs(k1 - ref[idx]) < 1e-12 * np.abs(ref).max()
        assert abs(k2 - ref[idx]) < 1e-12 * np.abs(ref).max()
        assert abs(got[idx] - k2) < 1e-12 * np.abs(ref).max()


def test_shifted_argument_errors():
    plan = su2.Plan(8, 1, "c128")
    with pytest.raises(su2.SU2Error):
        plan.beta_forward_shifted(depth=3)
    with pytest.raises(su2.SU2Error):
        plan.beta_forward_shifted(depth=2, block=3)
    with pytest.raises(su2.SU2Error):
        plan.beta_forward_shifted(depth=2, block=32)
    big = su2.Plan(128, 1, "c64")
    with pytest.raises(su2.SU2Error) as ei:
        big.beta_forward_shifted(depth=1)
    assert ei.value.status == 2
