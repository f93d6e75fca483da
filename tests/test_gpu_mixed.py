"""Mixed-bandlimit batches: persistent work-list kernels, HIP graph replay,
autotuned grid sizes.

Every signal of a mixed plan runs the same kernel bodies as a single-B plan,
so its results must be bit-identical to a batch-1 single-B plan of that
signal; the oracle then pins one signal per distinct bandlimit.
"""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2605_23923_amd as su2
import synth
from _errlog import record

pytestmark = pytest.mark.gpu

NPDT = {"c128": np.complex128, "c64": np.complex64, "c64_bf16x3": np.complex64}
TOL = {"c128": 1e-10, "c64": 1e-6, "c64_bf16x3": 1e-5}


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    return t.detach().cpu().numpy()


def _mixed_inputs(Bs, dtype, seed):
    rng = np.random.default_rng(seed)
    xs = [synth.samples_uniform(B, 1, seed=int(rng.integers(1 << 30)), dtype=NPDT[dtype])[0].reshape(-1) for B in Bs]
    cs = [synth.coeffs(B, 1, seed=int(rng.integers(1 << 30)), dtype=NPDT[dtype])[0] for B in Bs]
    return xs, cs


def _split(flat, offsets):
    return [flat[offsets[i]:offsets[i + 1]] for i in range(len(offsets) - 1)]


@pytest.mark.parametrize("dtype", ["c128", "c64", "c64_bf16x3"])
def test_mixed_bitwise_equals_single_plans(dtype):
    Bs = [16, 64, 24, 3, 32, 48, 16, 8, 64, 32]
    xs, cs = _mixed_inputs(Bs, dtype, 1)
    mp = su2.MixedPlan(Bs, dtype)
    k = mp.tuning()
    assert len(k) == 4 and all(v in (0, 1, 2, 3, 4, 6, 8) for v in k)
    x = _dev(np.concatenate(xs))
    c = _dev(np.concatenate(cs))
    f = _split(_host(mp.forward(x)), mp.coeff_offsets)
    i = _split(_host(mp.inverse(c)), mp.sample_offsets)
    a = _split(_host(mp.adjoint(c)), mp.sample_offsets)
    for s, B in enumerate(Bs):
        p = su2.Plan(B, 1, dtype)
        N = 2 * B
        assert np.array_equal(f[s], _host(p.forward(_dev(xs[s].reshape(1, N, N, N))))[0]), (s, B, "forward")
        assert np.array_equal(i[s], _host(p.inverse(_dev(cs[s].reshape(1, -1)))).reshape(-1)), (s, B, "inverse")
        assert np.array_equal(a[s], _host(p.adjoint(_dev(cs[s].reshape(1, -1)))).reshape(-1)), (s, B, "adjoint")
        p.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_mixed_matches_oracle_one_signal_per_bandlimit(dtype):
    Bs = [12, 24, 6, 12, 24, 32]
    xs, cs = _mixed_inputs(Bs, dtype, 2)
    mp = su2.MixedPlan(Bs, dtype)
    f = _split(_host(mp.forward(_dev(np.concatenate(xs)))), mp.coeff_offsets)
    inv = _split(_host(mp.inverse(_dev(np.concatenate(cs)))), mp.sample_offsets)
    rng = np.random.default_rng(3)
    seen = set()
    for s, B in enumerate(Bs):
        if B in seen:
            continue
        seen.add(B)
        C = oracle.num_coeffs(B)
        sel = rng.choice(C, min(C, 200), replace=False)
        ref = oracle.forward(B, xs[s].astype(np.complex128), sel)
        got = f[s][sel]
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        record(f"mixed forward B={B} {dtype} sampled", rel, np.max(np.abs(got - ref)) / np.max(np.abs(ref)),
               tol=TOL[dtype])
        assert rel <= TOL[dtype], (B, rel)
        pts = rng.choice((2 * B) ** 3, 100, replace=False)
        ref = oracle.inverse(B, cs[s].astype(np.complex128), pts)
        rel = np.linalg.norm(inv[s][pts] - ref) / np.linalg.norm(ref)
        record(f"mixed inverse B={B} {dtype} sampled", rel, np.max(np.abs(inv[s][pts] - ref)) / np.max(np.abs(ref)),
               tol=TOL[dtype])
        assert rel <= TOL[dtype], (B, rel)


def test_mixed_graph_replays_with_eager_work_between():
    """The call is captured once and replayed: replays interleaved with eager
    torch work and synchronisations all give the eager-launch result."""
    Bs = [16, 32, 24, 64]
    xs, _ = _mixed_inputs(Bs, "c64", 4)
    mp = su2.MixedPlan(Bs, "c64")
    x = _dev(np.concatenate(xs))
    out = torch.empty(mp.coeff_shape, dtype=torch.complex64, device="cuda")
    ref = None
    for rep in range(4):
        junk = torch.randn(1 << 20, device="cuda").cumsum(0)      # unrelated eager work
        out.zero_()
        mp.forward(x, out=out)
        torch.cuda.synchronize()
        got = _host(out).copy()
        if ref is None:
            ref = got
        assert np.array_equal(got, ref), rep
        del junk
    out2 = mp.forward(x)                                          # new buffers: new graph
    assert np.array_equal(_host(out2), ref)
    singles = _split(ref, mp.coeff_offsets)
    p = su2.Plan(64, 1, "c64")
    assert np.array_equal(singles[3], _host(p.forward(_dev(xs[3].reshape(1, 128, 128, 128))))[0])


def test_autotuner_choice_does_not_change_results():
    Bs = [16, 48, 32, 24]
    xs, cs = _mixed_inputs(Bs, "c64", 5)
    x = _dev(np.concatenate(xs))
    c = _dev(np.concatenate(cs))
    tuned = su2.MixedPlan(Bs, "c64")
    old = os.environ.get("SU2_AUTOTUNE")
    os.environ["SU2_AUTOTUNE"] = "0"
    try:
        plain = su2.MixedPlan(Bs, "c64")
    finally:
        if old is None:
            del os.environ["SU2_AUTOTUNE"]
        else:
            os.environ["SU2_AUTOTUNE"] = old
    assert plain.tuning() == [2, 2, 2, 2]
    assert np.array_equal(_host(tuned.forward(x)), _host(plain.forward(x)))
    assert np.array_equal(_host(tuned.adjoint(c)), _host(plain.adjoint(c)))


@pytest.mark.parametrize("dtype", ["c128", "c64", "c64_bf16x3"])
@pytest.mark.parametrize("kind", ["real", "so3"])
def test_mixed_real_and_so3_bitwise_equal_single_plans(kind, dtype):
    """Mixed real-signal and SO(3) plans: every signal equals a batch-1 plan of
    the same kind, bit for bit (half-spectrum rings at B = 8, 16, 64, generic
    rings at B = 12, 24)."""
    Bs = [16, 12, 64, 8, 24, 16, 64]
    rng = np.random.default_rng(41)
    kw = dict(real=True) if kind == "real" else dict(group="so3")
    mp = su2.MixedPlan(Bs, dtype, **kw)
    xs, cs = [], []
    for B in Bs:
        if kind == "real":
            xs.append(synth.samples_uniform(B, 1, seed=int(rng.integers(1 << 30))).real.astype(
                np.float64 if dtype == "c128" else np.float32).reshape(-1))
            cs.append(synth.coeffs(B, 1, seed=int(rng.integers(1 << 30)), dtype=NPDT[dtype])[0])
        else:
            xs.append(synth.samples_uniform(B, 1, seed=int(rng.integers(1 << 30)), dtype=NPDT[dtype])[0].reshape(-1))
            cs.append(synth.coeffs_so3(B, 1, seed=int(rng.integers(1 << 30)), dtype=NPDT[dtype])[0])
    f = _split(_host(mp.forward(_dev(np.concatenate(xs)))), mp.coeff_offsets)
    i = _split(_host(mp.inverse(_dev(np.concatenate(cs)))), mp.sample_offsets)
    a = _split(_host(mp.adjoint(_dev(np.concatenate(cs)))), mp.sample_offsets)
    def same(got, ref, what):
        diff = np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300)
        assert np.array_equal(got, ref), (what, f"max relative difference {diff:.3e}")

    for s_, B in enumerate(Bs):
        p = su2.Plan(B, 1, dtype, **kw)
        N = 2 * B
        same(f[s_], _host(p.forward(_dev(xs[s_].reshape(1, N, N, N))))[0], (s_, B, "forward"))
        same(i[s_], _host(p.inverse(_dev(cs[s_].reshape(1, -1)))).reshape(-1), (s_, B, "inverse"))
        same(a[s_], _host(p.adjoint(_dev(cs[s_].reshape(1, -1)))).reshape(-1), (s_, B, "adjoint"))
        p.close()


def test_pinned_grid_rejects_values_the_search_cannot_choose():
    """SU2_GRID must name four candidates (0, 1, 2, 3, 4, 6, 8): anything else
    is ignored and the plan keeps its defaults."""
    for bad in ("5,5,5,5", "1,2,3", "-1,0,0,0", "x"):
        with _env(SU2_AUTOTUNE="0", SU2_GRID=bad):
            mp = su2.MixedPlan([16, 24], "c64")
        assert mp.tuning() == [2, 2, 2, 2], bad
        mp.close()


@pytest.mark.parametrize("dtype", ["c128", "c64", "c64_bf16x3"])
def test_mixed_with_b128_groups(dtype):
    """B = 128 groups in a mixed plan run the single-B plan's N = 256 ring
    kernels (one pass in FP32, two passes in FP64) beside the work lists:
    every signal bit for bit equal to its single-B plan, and the B = 128
    signals to sampled oracle coefficients and points."""
    Bs = [128, 16, 128]
    xs, cs = _mixed_inputs(Bs, dtype, 12)
    with _env(SU2_AUTOTUNE="0"):
        mp = su2.MixedPlan(Bs, dtype)
    f = _split(_host(mp.forward(_dev(np.concatenate(xs)))), mp.coeff_offsets)
    i = _split(_host(mp.inverse(_dev(np.concatenate(cs)))), mp.sample_offsets)
    a = _split(_host(mp.adjoint(_dev(np.concatenate(cs)))), mp.sample_offsets)
    mp.close()
    for s, B in enumerate(Bs):
        N = 2 * B
        p = su2.Plan(B, 1, dtype)
        assert np.array_equal(f[s], _host(p.forward(_dev(xs[s].reshape(1, N, N, N))))[0]), (s, B, "forward")
        assert np.array_equal(i[s], _host(p.inverse(_dev(cs[s].reshape(1, -1)))).reshape(-1)), (s, B, "inverse")
        assert np.array_equal(a[s], _host(p.adjoint(_dev(cs[s].reshape(1, -1)))).reshape(-1)), (s, B, "adjoint")
        p.close()
    rng = np.random.default_rng(5)
    sel = rng.choice(oracle.num_coeffs(128), 6, replace=False)
    ref = oracle.forward(128, xs[2].astype(np.complex128), sel)
    rel = np.linalg.norm(f[2][sel] - ref) / np.linalg.norm(ref)
    assert rel <= TOL[dtype], ("forward", rel)
    pts = rng.choice(256 ** 3, 24, replace=False)
    ref = oracle.inverse(128, cs[2].astype(np.complex128), pts)
    rel = np.linalg.norm(i[2][pts] - ref) / np.linalg.norm(ref)
    assert rel <= TOL[dtype], ("inverse", rel)


def test_mixed_real_with_b128_group():
    """Real signals at B = 128 in a mixed plan (the N = 256 kernels with real
    samples in and the real part out) equal batch-1 real single-B plans bit
    for bit, beside a half-spectrum B = 16 signal."""
    Bs = [16, 128]
    rng = np.random.default_rng(17)
    xs = [synth.samples_uniform(B, 1, seed=int(rng.integers(1 << 30))).real.astype(np.float32).reshape(-1)
          for B in Bs]
    cs = [synth.coeffs(B, 1, seed=int(rng.integers(1 << 30)), dtype=np.complex64)[0] for B in Bs]
    with _env(SU2_AUTOTUNE="0"):
        mp = su2.MixedPlan(Bs, "c64", real=True)
    f = _split(_host(mp.forward(_dev(np.concatenate(xs)))), mp.coeff_offsets)
    i = _split(_host(mp.inverse(_dev(np.concatenate(cs)))), mp.sample_offsets)
    mp.close()
    for s, B in enumerate(Bs):
        p = su2.Plan(B, 1, "c64", real=True)
        N = 2 * B
        assert np.array_equal(f[s], _host(p.forward(_dev(xs[s].reshape(1, N, N, N))))[0]), (B, "forward")
        assert np.array_equal(i[s], _host(p.inverse(_dev(cs[s].reshape(1, -1)))).reshape(-1)), (B, "inverse")
        p.close()


class _env:
    """Set environment variables for the plan creations inside the block."""

    def __init__(self, **kv):
        self.kv = kv

    def __enter__(self):
        self.old = {k: os.environ.get(k) for k in self.kv}
        os.environ.update(self.kv)

    def __exit__(self, *exc):
        for k, v in self.old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


# groups of at most 16 signals and larger ones, every B class of the contraction
SHAPE_BS = [8] * 3 + [24] * 20 + [32] * 5 + [48] * 17 + [64] * 2


@pytest.mark.parametrize("dtype", ["c128", "c64", "c64_bf16x3"])
def test_pinned_grids_bitwise_equal_defaults(dtype):
    """SU2_GRID pins the four work-list grids: one workgroup per task (0) and
    the smallest persistent grid (1, every workgroup walking many tasks) give
    the default grids' results bit for bit in all three directions, with the
    register-resident and the generic ring lists and both contraction lists."""
    Bs = [16, 48, 32, 24, 64, 8, 32, 48]
    xs, cs = _mixed_inputs(Bs, dtype, 9)
    x = _dev(np.concatenate(xs))
    c = _dev(np.concatenate(cs))
    with _env(SU2_AUTOTUNE="0"):
        ref = su2.MixedPlan(Bs, dtype)
    want = [_host(ref.forward(x)), _host(ref.inverse(c)), _host(ref.adjoint(c))]
    ref.close()
    for grid in ("0,0,0,0", "1,1,1,1", "0,1,0,1"):
        with _env(SU2_AUTOTUNE="0", SU2_GRID=grid):
            mp = su2.MixedPlan(Bs, dtype)
        assert mp.tuning() == [int(v) for v in grid.split(",")]
        got = [_host(mp.forward(x)), _host(mp.inverse(c)), _host(mp.adjoint(c))]
        mp.close()
        for name, a, b in zip(("forward", "inverse", "adjoint"), got, want):
            assert np.array_equal(a, b), (grid, name)


def test_tile_shapes_defaults_reported():
    with _env(SU2_AUTOTUNE="0"):
        mp = su2.MixedPlan(SHAPE_BS, "c64")
        md = su2.MixedPlan(SHAPE_BS, "c128")
        mb = su2.MixedPlan(SHAPE_BS, "c64_bf16x3")
    counts = {B: SHAPE_BS.count(B) for B in set(SHAPE_BS)}
    assert [s[0] for s in mp.tile_shapes()] == sorted(counts)
    for B, f, i, kc in mp.tile_shapes():
        w = 16 if counts[B] <= 16 else 32
        assert (f, i, kc) == (w, w, 4), B
    assert all(s[1:] == (16, 16, 8) for s in md.tile_shapes())
    for B, f, i, kc in mb.tile_shapes():
        assert (f, i, kc) == (16, 16 if counts[B] <= 16 else 32, 32), B


@pytest.mark.parametrize("dtype,shapes", [
    ("c64", "4,16,16"), ("c64", "8,32,32"), ("c64", "8,16,32"), ("c64", "4,32,16"),
    ("c128", "4,16,16"), ("c128", "8,16,16"),
    ("c64_bf16x3", "32,16,16"), ("c64_bf16x3", "32,16,32"),
])
def test_pinned_tile_shapes_bitwise_equal_default(dtype, shapes):
    """Every tile shape gives the default shape's bits in all three directions
    (sums over beta run in node order whatever the tile), and is reported."""
    xs, cs = _mixed_inputs(SHAPE_BS, dtype, 7)
    x = _dev(np.concatenate(xs))
    c = _dev(np.concatenate(cs))
    with _env(SU2_AUTOTUNE="0"):
        ref = su2.MixedPlan(SHAPE_BS, dtype)
    with _env(SU2_AUTOTUNE="0", SU2_TILE_SHAPES=shapes):
        mp = su2.MixedPlan(SHAPE_BS, dtype)
    kc, fw, iw = (int(v) for v in shapes.split(","))
    for B, f, i, k in mp.tile_shapes():
        assert k == kc and i == iw, (B, k, i)
        assert f == (16 if dtype != "c64" else fw), (B, f)
    for fn in ("forward", "inverse", "adjoint"):
        a = ref.forward(x) if fn == "forward" else getattr(ref, fn)(c)
        b = mp.forward(x) if fn == "forward" else getattr(mp, fn)(c)
        assert np.array_equal(_host(a), _host(b)), fn


# 65-128 degrees in both tile widths: 17 signals of B = 72 (32-signal tiles)
# and 2 of B = 96 (16-signal tiles).  Both bodies in one kernel would take 195
# VGPRs in the FP32 forward, so each width is a launch of its own there (and
# in the inverse), the class being split in two runs.
SPLIT_BS = [72] * 17 + [96] * 2


def test_split_width_runs_bitwise_equal_single_width():
    """The default tile shapes of SPLIT_BS (one run per width in the classes
    of 65-128 degrees) give the bits of every group in one width, 16 or 32
    signals, in all three directions."""
    xs, cs = _mixed_inputs(SPLIT_BS, "c64", 11)
    x = _dev(np.concatenate(xs))
    c = _dev(np.concatenate(cs))
    with _env(SU2_AUTOTUNE="0"):
        ref = su2.MixedPlan(SPLIT_BS, "c64")
    assert [tuple(s) for s in ref.tile_shapes()] == [(72, 32, 32, 4), (96, 16, 16, 4)]
    want = [_host(ref.forward(x)), _host(ref.inverse(c)), _host(ref.adjoint(c))]
    ref.close()
    for shapes in ("4,16,16", "4,32,32"):
        with _env(SU2_AUTOTUNE="0", SU2_TILE_SHAPES=shapes):
            mp = su2.MixedPlan(SPLIT_BS, "c64")
        got = [_host(mp.forward(x)), _host(mp.inverse(c)), _host(mp.adjoint(c))]
        mp.close()
        for name, a, b in zip(("forward", "inverse", "adjoint"), got, want):
            assert np.array_equal(a, b), (shapes, name)


def test_autotuned_tile_shapes_valid_and_cached(tmp_path):
    """The search picks a valid shape per group and changes no result; a fresh
    process reads the choice back from the disk cache instead of searching."""
    cache = tmp_path / "tune.txt"
    xs, cs = _mixed_inputs(SHAPE_BS, "c64", 8)
    x = _dev(np.concatenate(xs))
    c = _dev(np.concatenate(cs))
    with _env(SU2_AUTOTUNE_CACHE=str(cache), SU2_TILE_SHAPES="4,16,32"):
        pinned = su2.MixedPlan(SHAPE_BS, "c64")       # pinned shapes: a cache key of their own
    assert pinned.tile_shapes() == [(B, 16, 32, 4) for B in sorted(set(SHAPE_BS))]
    with _env(SU2_AUTOTUNE_CACHE=str(cache)):
        tuned = su2.MixedPlan(SHAPE_BS, "c64")
    shapes = tuned.tile_shapes()
    assert all(f in (16, 32) and i in (16, 32) and k in (4, 8) for _, f, i, k in shapes)
    assert len(set(k for *_, k in shapes)) == 1
    lines = cache.read_text().splitlines()
    assert any("pinned4,16,32" in ln for ln in lines)
    with _env(SU2_AUTOTUNE="0"):
        plain = su2.MixedPlan(SHAPE_BS, "c64")
    for fn in ("forward", "adjoint"):
        a = plain.forward(x) if fn == "forward" else plain.adjoint(c)
        b = tuned.forward(x) if fn == "forward" else tuned.adjoint(c)
        assert np.array_equal(_host(a), _host(b)), fn
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import paper_2605_23923_amd as su2; "
            f"mp = su2.MixedPlan({SHAPE_BS!r}, 'c64'); print(mp.tile_shapes(), mp.tuning())")
    env = dict(os.environ, SU2_AUTOTUNE_CACHE=str(cache), PYTHONPATH=root)
    env.pop("SU2_TILE_SHAPES", None)
    env.pop("SU2_AUTOTUNE", None)
    out = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip() == f"{shapes} {tuned.tuning()}"
    assert cache.read_text().splitlines() == lines       # nothing searched, nothing appended


def test_mixed_batch_configuration_320_signals():
    """256 signals at B = 32 plus 64 signals with B drawn from {16, 24, 32, 48, 64}
    (seed 33), FP32, one mixed plan; sampled signals against batch-1 plans
    (bitwise) and one signal per distinct B against the oracle."""
    Bs = [32] * 256 + synth.bandlimits_mixed(64, seed=33)
    mp = su2.MixedPlan(Bs, "c64")
    rng = np.random.default_rng(34)
    xs = [synth.samples_uniform(B, 1, seed=1000 + s, dtype=np.complex64)[0].reshape(-1) for s, B in enumerate(Bs)]
    f = _split(_host(mp.forward(_dev(np.concatenate(xs)))), mp.coeff_offsets)
    checked = set()
    for s in list(rng.choice(len(Bs), 6, replace=False)) + [256 + i for i in range(64)]:
        B = Bs[s]
        if s >= 256 and B in checked:
            continue
        p = su2.Plan(B, 1, "c64")
        N = 2 * B
        assert np.array_equal(f[s], _host(p.forward(_dev(xs[s].reshape(1, N, N, N))))[0]), (s, B)
        p.close()
        if s >= 256:
            checked.add(B)
            C = oracle.num_coeffs(B)
            sel = rng.choice(C, 64, replace=False)
            ref = oracle.forward(B, xs[s].astype(np.complex128), sel)
            rel = np.linalg.norm(f[s][sel] - ref) / np.linalg.norm(ref)
            record(f"mixed 320-signal forward B={B} c64 sampled", rel,
                   np.max(np.abs(f[s][sel] - ref)) / np.max(np.abs(ref)), tol=TOL["c64"])
            assert rel <= TOL["c64"], (B, rel)
    assert checked == set(Bs[256:])
