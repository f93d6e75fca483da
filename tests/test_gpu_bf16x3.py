"""GPU parity of the split-bfloat16 beta contraction (mode c64_bf16x3).

Tolerance: 1e-5 normwise relative error (the target the split-precision mode
is specified to).  Each FP32 operand is carried as hi + lo with
|x - hi - lo| <= 2^-16 |x|; the three products drop lo*lo (<= 2^-16 |ab|), so a
single product is off by at most ~3 * 2^-16 = 4.6e-5 relative and the rounding
errors of the N-term (or L-term) sums average out, leaving an expected
normwise error of a few 1e-6 (observed on MI355X: 2.0e-6 to 5.5e-6 at every
B, worst element at most 1.9x the normwise figure).  The worst element is
allowed 10x the normwise bound.  The FFT stage is the FP32 one.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_23923_amd as su2
import synth
from _errlog import record

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def _rel(got, ref):
    got = np.asarray(got).reshape(-1)
    ref = np.asarray(ref).reshape(-1)
    return np.linalg.norm(got - ref) / np.linalg.norm(ref), np.max(np.abs(got - ref)) / np.max(np.abs(ref))


@pytest.mark.parametrize("B,batch", [(1, 3), (2, 3), (3, 3), (4, 3), (8, 3), (16, 3), (24, 3),
                                     # batches above 16 take the 32-signal inverse tiles (here one partial)
                                     (8, 21), (16, 40)])
def test_bf16x3_matches_oracle(B, batch):
    x = synth.samples_uniform(B, batch, seed=400 + B, dtype=np.complex64)
    c = synth.coeffs(B, batch, seed=500 + B, dtype=np.complex64)
    plan = su2.Plan(B, batch, "c64_bf16x3")
    gf = _host(plan.forward(_dev(x)))
    gi = _host(plan.inverse(_dev(c)))
    ga = _host(plan.adjoint(_dev(c)))
    N = 2 * B
    pts = None if B <= 16 else np.random.default_rng(B).choice(N ** 3, 300, replace=False)
    for b in (range(batch) if batch <= 3 else (0, batch // 2, batch - 1)):
        rf = oracle.forward(B, x[b])
        ri = oracle.inverse(B, c[b], pts)
        ra = oracle.adjoint(B, c[b], pts)
        gib = gi[b].reshape(-1) if pts is None else gi[b].reshape(-1)[pts]
        gab = ga[b].reshape(-1) if pts is None else ga[b].reshape(-1)[pts]
        for got, ref, what in ((gf[b], rf, "forward"), (gib, ri, "inverse"), (gab, ra, "adjoint")):
            rel, worst = _rel(got, ref)
            print(f"bf16x3 {what} B={B} s{b}: rel {rel:.3e} worst {worst:.3e}", flush=True)
            record(f"bf16x3 {what} B={B} batch {batch} s{b}", rel, worst, tol=TOL)
            assert rel <= TOL and worst <= 10 * TOL, f"{what} B={B}: rel {rel:.3e} worst {worst:.3e}"


def _stratified_coeffs(B, count, rng):
    """Coefficient indices covering every 2l, with the extreme m, n of each block."""
    sel = []
    for tl in range(B):
        base = oracle.coeff_index(tl, -tl, -tl)
        sel += [base, base + (tl + 1) ** 2 - 1]
    extra = rng.choice(oracle.num_coeffs(B), count, replace=False)
    return np.unique(np.concatenate([np.array(sel), extra]))


def test_bf16x3_b64_batch32_matches_oracle():
    """B = 64, batch 32 in split BF16: the shape and launch configuration the
    benchmark times (two row tiles per pair in the forward contraction, two
    16-signal tiles; one 32-signal tile in the inverse).  Forward on sampled
    coefficients of signals in both signal tiles, inverse and adjoint at
    sampled sample points, all against the oracle, 1e-5 normwise."""
    B, batch = 64, 32
    N = 2 * B
    rng = np.random.default_rng(6464)
    plan = su2.Plan(B, batch, "c64_bf16x3")
    x = synth.samples_uniform(B, batch, seed=641, dtype=np.complex64)
    gf = _host(plan.forward(_dev(x)))
    assert np.all(np.isfinite(gf))
    sel = _stratified_coeffs(B, 64, rng)
    for b in (0, 15, 16, 31):
        ref = oracle.forward(B, x[b], sel)
        rel, worst = _rel(gf[b][sel], ref)
        print(f"bf16x3 forward B=64 batch 32 s{b}: rel {rel:.3e} worst {worst:.3e}", flush=True)
        record(f"bf16x3 forward B=64 batch 32 s{b}", rel, worst, tol=TOL)
        assert rel <= TOL and worst <= 10 * TOL, f"forward s{b}: rel {rel:.3e} worst {worst:.3e}"
    del x
    c = synth.coeffs(B, batch, seed=642, spectrum="decay", dtype=np.complex64)
    gi = _host(plan.inverse(_dev(c)))
    ga = _host(plan.adjoint(_dev(c)))
    pts = np.concatenate([rng.choice(N ** 3, 60, replace=False), [0, N ** 3 - 1, N * N * (N - 1)]])
    for b in (0, 16, 31):
        for got, ref, what in ((gi[b].reshape(-1)[pts], oracle.inverse(B, c[b], pts), "inverse"),
                               (ga[b].reshape(-1)[pts], oracle.adjoint(B, c[b], pts), "adjoint")):
            rel, worst = _rel(got, ref)
            print(f"bf16x3 {what} B=64 batch 32 s{b}: rel {rel:.3e} worst {worst:.3e}", flush=True)
            record(f"bf16x3 {what} B=64 batch 32 s{b}", rel, worst, tol=TOL)
            assert rel <= TOL and worst <= 10 * TOL, f"{what} s{b}: rel {rel:.3e} worst {worst:.3e}"


def _per_two_l(got, ref, B, gnorm):
    """Per 2l: max |error|, error norm of the block relative to the block's
    reference norm, and relative to the signal's global norm."""
    tl_of = synth.two_l_of_index(B)
    rows = []
    for tl in range(B):
        m = tl_of == tl
        err = got[m] - ref[m]
        rows.append([tl, float(np.max(np.abs(err))), float(np.linalg.norm(err) / np.linalg.norm(ref[m])),
                     float(np.linalg.norm(err) / gnorm)])
    return rows


def _print_table(title, rows):
    print(title)
    print(" 2l  max|err|     block rel      rel to global norm")
    for tl, mx, brel, grel in rows:
        if tl < 8 or tl % 16 == 15:
            print(f"{tl:4d}  {mx:.3e}   {brel:.3e}      {grel:.3e}")


def test_bf16x3_b128_batch16_spiked_precision():
    """B = 128, batch 16, 256^3 grid, split BF16, a flat CN(0,1) spectrum whose
    blocks 2l <= 3 are scaled to 1e-6 (the spiked precision workload).

    Forward: FP32 samples synthesised from the coefficients in FP64 (then
    rounded); compared per 2l with the seeded coefficients themselves (exact
    quadrature; the samples carry FP32 rounding, about 1e-7 relative) and with
    the oracle's direct sum on the same FP32 samples for sampled coefficients
    of every 2l.

    Inverse and adjoint: against the oracle at sampled points of three signals
    (1e-5 normwise); and per 2l, by analysing the split-BF16 output with the
    FP64 forward (whose parity with the oracle at this size is tested
    separately): forward(inverse(c)) = c and forward(adjoint(c) / W_k) =
    c / (2l + 1) hold exactly in exact arithmetic, so the difference per block
    is the part of the output error that lies in degree 2l.

    The 1e-5 bound applies normwise over each signal and to every block that
    is not spiked; the 1e-6 blocks sit below the absolute error floor of
    ~1e-5 x the signal scale and are reported only.  Every per-2l table is
    written to the error log."""
    B, batch = 128, 16
    N = 2 * B
    c = synth.coeffs(B, batch, seed=4, spike_tl=(0, 1, 2, 3), spike_scale=1e-6)
    ref_plan = su2.Plan(B, batch, "c128")
    x64 = ref_plan.inverse(_dev(c))
    x32 = x64.to(torch.complex64)
    del x64
    torch.cuda.empty_cache()
    plan = su2.Plan(B, batch, "c64_bf16x3")
    got = _host(plan.forward(x32))
    worst_signal = 0.0
    for b in range(batch):
        rel, _ = _rel(got[b], c[b])
        worst_signal = max(worst_signal, rel)
    print(f"B=128 batch 16 bf16x3 forward: worst per-signal normwise rel {worst_signal:.3e}")
    record("bf16x3 forward B=128 batch 16 spiked, vs seeded coefficients (worst signal)", worst_signal, 0.0, tol=TOL)
    gnorm = np.linalg.norm(c[0])
    rows = _per_two_l(got[0], c[0], B, gnorm)
    _print_table("forward, signal 0, vs seeded coefficients", rows)
    record("bf16x3 forward B=128 batch 16 spiked, per 2l (signal 0)", max(r[3] for r in rows), 0.0, per_2l=rows)
    bad = [(r[0], r[2]) for r in rows if r[0] > 3 and r[2] > TOL]
    assert worst_signal <= TOL
    assert not bad, f"non-spiked forward blocks above {TOL}: {bad[:5]}"
    # oracle on the same FP32 samples, sampled coefficients of every 2l
    xs0 = x32[0].cpu().numpy().astype(np.complex128)
    del x32
    torch.cuda.empty_cache()
    rng = np.random.default_rng(128)
    sel = []
    for tl in range(0, B, 3):
        base = oracle.coeff_index(tl, -tl, -tl)
        sel.append(base + int(rng.integers(0, (tl + 1) ** 2)))
    sel = np.array(sel)
    ref = oracle.forward(B, xs0, sel)
    err = np.abs(got[0][sel] - ref)
    print(f"oracle (sampled, {sel.size} coefficients): max abs err {err.max():.3e}, "
          f"max |ref| {np.abs(ref).max():.3e}")
    record("bf16x3 forward B=128 batch 16 spiked, oracle sampled coefficients (max abs err / coefficient rms)",
           err.max() / (gnorm / np.sqrt(c[0].size)), 0.0)
    assert err.max() <= TOL * gnorm / np.sqrt(c[0].size) * 30
    del got, xs0

    # inverse and adjoint
    cd = _dev(c.astype(np.complex64))
    _, _, _, W = oracle.grid(B)
    Wd = torch.from_numpy(np.asarray(W, dtype=np.float64)).to("cuda").view(1, N, 1, 1)
    pts = np.concatenate([rng.choice(N ** 3, 24, replace=False), [0, N ** 3 - 1]])
    for what in ("inverse", "adjoint"):
        xo = plan.inverse(cd) if what == "inverse" else plan.adjoint(cd)
        host = xo.cpu().numpy()
        for b in (0, 7, 15):
            r = (oracle.inverse if what == "inverse" else oracle.adjoint)(B, c[b], pts)
            rel, worst = _rel(host[b].reshape(-1)[pts].astype(np.complex128), r)
            print(f"bf16x3 {what} B=128 batch 16 spiked s{b}: rel {rel:.3e} worst {worst:.3e}", flush=True)
            record(f"bf16x3 {what} B=128 batch 16 spiked s{b}", rel, worst, tol=TOL)
            assert rel <= TOL and worst <= 10 * TOL, f"{what} s{b}: rel {rel:.3e} worst {worst:.3e}"
        del host
        x128 = xo.to(torch.complex128)
        del xo
        torch.cuda.empty_cache()
        if what == "adjoint":
            x128 = x128 / Wd
        back = _host(ref_plan.forward(x128))
        del x128
        torch.cuda.empty_cache()
        target = c if what == "inverse" else c / (synth.two_l_of_index(B) + 1.0)
        worst_signal = max(_rel(back[b], target[b])[0] for b in range(batch))
        print(f"B=128 batch 16 bf16x3 {what}, analysed in FP64: worst per-signal normwise rel {worst_signal:.3e}")
        record(f"bf16x3 {what} B=128 batch 16 spiked, FP64 analysis (worst signal)", worst_signal, 0.0, tol=TOL)
        rows = _per_two_l(back[0], target[0], B, np.linalg.norm(target[0]))
        _print_table(f"{what}, signal 0, analysed by the FP64 forward", rows)
        record(f"bf16x3 {what} B=128 batch 16 spiked, per 2l (signal 0, FP64 analysis)", max(r[3] for r in rows),
               0.0, per_2l=rows)
        assert worst_signal <= TOL
        bad = [(r[0], r[2]) for r in rows if r[0] > 3 and r[2] > TOL]
        assert not bad, f"non-spiked {what} blocks above {TOL}: {bad[:5]}"
    ref_plan.close()
    plan.close()
