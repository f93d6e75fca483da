#!/usr/bin/env python3
"""Throughput of the separated SU(2) Fourier transform on one MI355X.

Workload: bandlimit B = 64 (128^3 Euler grid), batch of 32 signals, inputs from
seeded complex Gaussian bandlimited coefficients with variance (2l+1)^-2
(the samples are synthesised from them once, before timing).  One step runs
the whole transform chain on the batch: forward (ring FFT + beta contraction),
inverse (beta synthesis + inverse ring FFT) and adjoint (the same two kernels
with the quadrature weights), i.e. 3 x 32 single-signal transforms.

Printed: one JSON line.  `value` = single-signal transforms per second (each
forward, inverse or adjoint of one signal counts as one), from the wall clock
around the K timed steps (bracketed by device synchronisation).  Every kernel
is bracketed by HIP events on the stream it runs on; `roofline` reports the
kernel with the largest share of the step against the HBM peak, with its
algorithmic bytes per launch.  `cpu_baseline` times the CPU oracle (direct
quadrature sum) on a bounded sample of the same forward workload on all host
cores (`cpu_baseline_1core`: on one), and
`cpu_fft_baseline` a plain CPU FFT-based separated transform (float64) beside it
(`cpu_fft_baselines`: float64 and float32, forward and inverse).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12            # B/s, MI355X HBM3E
MFMA_PEAK = {"c128": 78.6e12, "c64": 157.3e12, "c64_bf16x3": 2.5e15}   # dense FP64 / FP32 / BF16
DTYPE_NAME = {"c128": "f64", "c64": "f32", "c64_bf16x3": "f32+bf16x3"}
# (B, batch) of the shapes bench.py can time on their own: stage by stage, or
# (mixed_320: 320 signals of mixed bandlimits) the whole step
WORKLOADS = {"b64_batch32": (64, 32), "b128_batch16": (128, 16), "mixed_320": (None, 320)}
STAGES = ["ring_forward", "beta_forward", "beta_inverse", "ring_inverse", "beta_adjoint", "ring_adjoint"]
# a mode is a precision ("c128", "c64", "c64_bf16x3"), optionally with "_otf"
# (Wigner-d values generated inside the contraction kernels instead of stored)
# or "_real" (real signals: real samples, half of the pairs contracted)
# or "_so3" (the transform on SO(3): integer degrees only, same grid size)


def base_mode(mode: str) -> str:
    for suffix in ("_otf", "_real", "_so3"):
        if mode.endswith(suffix):
            return mode[: -len(suffix)]
    return mode


def kernel_name(stage: str, mode: str) -> str:
    """Name of the kernel that runs `stage` at B=64, as rocprofv3 lists it (template type kept)."""
    t = "double" if base_mode(mode) == "c128" else "float"
    if stage.startswith("ring"):
        if stage != "ring_forward" and t == "double":
            return "ring_inverse_fast_pair<double>"   # FP64 inverse: two rings per workgroup
        return f"ring_{'forward' if stage == 'ring_forward' else 'inverse'}_fast<{t}>"
    kind = "forward" if stage == "beta_forward" else "inverse"
    if mode == "c64_bf16x3":
        return f"beta_{kind}_bf16x3_kernel"
    if mode.endswith("_otf"):
        return f"beta_{kind}_otf_kernel<{t}>"
    return f"beta_{kind}_kernel<{t}>"


def retained_pairs(B: int) -> int:
    return 2 * B * B - 2 * B + 1


def num_coeffs(B: int, mode: str) -> int:
    """Coefficients (= table rows) per signal: every 2l < B, or integer l only for SO(3)."""
    if mode.endswith("_so3"):
        L = (B - 1) // 2 + 1
        return L * (2 * L - 1) * (2 * L + 1) // 3
    return B * (B + 1) * (2 * B + 1) // 6


def table_bytes(B: int, mode: str) -> int:
    """Table bytes a contraction launch reads: the stored table, or the
    scalars of the generated one (3 recurrence coefficients per degree, a
    seed constant per pair, 3 values per node, all FP64).  The stored table
    is symmetry-reduced: the pairs (m, n) and (-m, -n) share one column up to
    the sign (-1)^{m-n}, so it holds (C + C0) / 2 columns of 2B nodes, C0
    being the coefficients with m = n = 0 (one per integer l)."""
    C = num_coeffs(B, mode)
    if mode.endswith("_otf"):
        return 8 * (3 * C + retained_pairs(B) + 3 * 2 * B)
    es = {"c128": 8, "c64": 4, "c64_bf16x3": 4}[base_mode(mode)]
    C0 = (B - 1) // 2 + 1
    return (C + C0) // 2 * 2 * B * es


def algorithmic_bytes(stage: str, B: int, batch: int, mode: str) -> int:
    """Compulsory HBM bytes of one launch: inputs read once, outputs written once."""
    N = 2 * B
    cb = 16 if base_mode(mode) == "c128" else 8
    C = B * (B + 1) * (2 * B + 1) // 6
    ring = N ** 3 * cb                       # one signal's samples
    spec = retained_pairs(B) * N * cb        # one signal's retained ring spectra
    coef = C * cb
    if mode.endswith("_so3"):
        # every sample read; spectra of the (2L - 1)^2 integer pairs; the
        # integer-degree coefficients and table rows
        L = (B - 1) // 2 + 1
        spec = (2 * L - 1) ** 2 * N * cb
        coef = num_coeffs(B, mode) * cb
        if stage.startswith("ring"):
            return batch * (ring + spec)
        return batch * (spec + coef) + table_bytes(B, mode)
    if mode.endswith("_real"):
        # real samples; spectra of the (P + 1) / 2 pairs with 2m >= 0 (mirrors
        # excluded); every coefficient written (forward) or read (inverse);
        # the table columns of those pairs (one per (m, n), (-m, -n) couple:
        # the whole symmetry-reduced table)
        ring = N ** 3 * cb // 2
        spec = (retained_pairs(B) + 1) // 2 * N * cb
        if stage.startswith("ring"):
            return batch * (ring + spec)
        return batch * (spec + coef) + table_bytes(B, base_mode(mode))
    if stage.startswith("ring"):
        return batch * (ring + spec)
    return batch * (spec + coef) + table_bytes(B, mode)


def step_bytes(counts: dict, mode: str) -> int:
    """Algorithmic HBM bytes of one forward + inverse + adjoint step over a
    batch given as {bandlimit: signals}: each direction is a ring stage and a
    contraction stage per bandlimit (the table read once per stage and B)."""
    per_dir = sum(algorithmic_bytes("ring_forward", B, n, mode) + algorithmic_bytes("beta_forward", B, n, mode)
                  for B, n in counts.items())
    return 3 * per_dir


def step_hbm_frac(counts: dict, mode: str, ms_per_step: float) -> float:
    """step_bytes over the step time, against the 8 TB/s peak."""
    return round(step_bytes(counts, mode) / (ms_per_step * 1e-3) / HBM_PEAK, 4)


def useful_flops(stage: str, B: int, batch: int, mode: str = "c64") -> float:
    """Useful real flops of a beta contraction: 4 per (l, m, n, k, signal)."""
    N = 2 * B
    return 4.0 * N * num_coeffs(B, mode) * batch if stage.startswith("beta") else 0.0


def shifted_depth1_flops(B: int, batch: int) -> float:
    """Flops of the depth-1 shifted contraction: fhat(l0 + rho) sums
    A_{rho-1} s^{Lb} + B_{rho-1} s^{Lb-1} over the nodes, two real-times-complex
    multiply-adds (8 flops) per (coefficient, node, signal)."""
    return 8.0 * 2 * B * num_coeffs(B, "c64") * batch


# sources of the kernels the B = 64 chain launches (the counter summaries in
# profiles/ are valid only for the digest they were taken at)
MEASURED_SOURCES = ["su2fft_internal.h", "su2fft_ring_fast.hip", "su2fft_beta.hip", "su2fft_beta_bf16.hip"]


def source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2605_23923_amd", "csrc")
    for fn in MEASURED_SOURCES:
        with open(os.path.join(csrc, fn), "rb") as fh:
            h.update(fn.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, mode: str, digest: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    ent = data.get(f"{kernel}:{mode}")
    if not ent or ent.get("source_digest") != digest:
        return None
    return ent.get("bytes_per_launch")


def run_mode(mode: str, B: int, batch: int, steps: int, warmup: int, timed_steps: bool):
    import torch

    import paper_2605_23923_amd as su2
    import synth

    # plan creation (grid, pair order, Wigner-d tables generated on the GPU,
    # workspace) is set-up, outside the timed steps; reported on its own
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    plan = su2.Plan(B, batch, base_mode(mode), tables="on_the_fly" if mode.endswith("_otf") else "stored",
                    real=mode.endswith("_real"), group="so3" if mode.endswith("_so3") else "su2")
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - tp0) * 1e3
    np_dt = "complex128" if base_mode(mode) == "c128" else "complex64"
    if mode.endswith("_so3"):
        c_host = synth.coeffs_so3(B, batch, seed=2, spectrum="decay").astype(np_dt)
    else:
        c_host = synth.coeffs(B, batch, seed=2, spectrum="decay").astype(np_dt)
    coeffs = torch.from_numpy(c_host).to("cuda")
    samples = plan.inverse(coeffs)                       # input synthesis, not timed
    c_out = torch.empty_like(coeffs)
    x_out = torch.empty_like(samples)
    a_out = torch.empty_like(samples)
    args = {"ring_forward": (samples, None), "beta_forward": (None, c_out), "beta_inverse": (coeffs, None),
            "ring_inverse": (None, x_out), "beta_adjoint": (coeffs, None), "ring_adjoint": (None, a_out)}

    def step(evs=None):
        for i, st in enumerate(STAGES):
            if evs is not None:
                evs[i].record()
            plan.run_stage(st, *args[st])
        if evs is not None:
            evs[len(STAGES)].record()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(STAGES) + 1)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        step(events[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage_ms = {st: 0.0 for st in STAGES}
    for s in range(steps):
        for i, st in enumerate(STAGES):
            stage_ms[st] += events[s][i].elapsed_time(events[s][i + 1]) / steps
    ms_per_step = (t1 - t0) * 1e3 / steps
    out = {
        "plan_ms": plan_ms,
        "ms_per_step": ms_per_step,
        "transforms_per_s": 3 * batch / (ms_per_step * 1e-3),
        "forward_per_s": batch / ((stage_ms["ring_forward"] + stage_ms["beta_forward"]) * 1e-3),
        "inverse_per_s": batch / ((stage_ms["beta_inverse"] + stage_ms["ring_inverse"]) * 1e-3),
        "adjoint_per_s": batch / ((stage_ms["beta_adjoint"] + stage_ms["ring_adjoint"]) * 1e-3),
        "stage_ms": {k: round(v, 5) for k, v in stage_ms.items()},
        "stage_hbm_frac": {k: round(algorithmic_bytes(k, B, batch, mode) / (v * 1e-3) / HBM_PEAK, 4)
                           for k, v in stage_ms.items()},
        "beta_mfma_useful_frac": {k: round(useful_flops(k, B, batch, mode) / (stage_ms[k] * 1e-3) /
                                           MFMA_PEAK[base_mode(mode)], 5)
                                  for k in STAGES if k.startswith("beta")},
    }
    plan.close()
    del samples, coeffs, c_out, x_out, a_out
    torch.cuda.empty_cache()
    return out


def run_whole(make_plan, x, c, steps: int, warmup: int, batch: int):
    """Time forward + inverse + adjoint through the public calls (no stage split)."""
    import torch

    plan = make_plan()
    y = plan.forward(x)
    xi = plan.inverse(c)
    xa = plan.adjoint(c)

    def step():
        plan.forward(x, out=y)
        plan.inverse(c, out=xi)
        plan.adjoint(c, out=xa)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    info = {"ms_per_step": round(dt * 1e3, 4), "transforms_per_s": round(3 * batch / dt, 2)}
    if hasattr(plan, "tuning"):
        info["workgroups_per_cu"] = plan.tuning()
        info["tile_shapes_B_fwd_inv_kc"] = [list(s) for s in plan.tile_shapes()]
    plan.close()
    return info


def run_separate(make_plan, x, c, steps: int, warmup: int):
    """Forward and inverse of one plan timed apart (HIP events, mean over steps)."""
    import torch

    plan = make_plan()
    y = plan.forward(x)
    xi = plan.inverse(c)
    res = {}
    for name, fn in (("forward_ms", lambda: plan.forward(x, out=y)), ("inverse_ms", lambda: plan.inverse(c, out=xi))):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        e1.synchronize()
        res[name] = round(e0.elapsed_time(e1) / steps, 4)
    plan.close()
    return res


def shifted_forms(steps: int):
    """The forward contraction at B=64 batch 32 (c64 plan) in its three forms:
    the table contraction on the matrix cores, and the shifted-recurrence
    (divide-and-conquer) form at depth 1 and at depth 2 with coarse step 16
    (FP64 matrix cores, the shifted polynomials generated in FP64 on the
    vector ALUs), and at depth 2 with coarse step 4 (FP64 vector ALUs).  The
    matrix-core forms are priced by their contraction: two real-times-complex
    multiply-adds per (coefficient, node, signal), one against each stored
    product, i.e. 8 N C(B) flops per signal, against the dense FP64
    matrix-core peak."""
    import numpy as np
    import torch

    import paper_2605_23923_amd as su2
    import synth

    B, batch = 64, 32
    plan = su2.Plan(B, batch, "c64")
    x = torch.from_numpy(synth.samples_uniform(B, batch, seed=1, dtype=np.complex64)).to("cuda")
    out = torch.empty(plan.coeff_shape, dtype=plan.torch_dtype, device="cuda")
    plan.run_stage("ring_forward", x, None)
    res = {}
    for name, fn in (("table_ms", lambda: plan.run_stage("beta_forward", None, out)),
                     ("shifted_depth1_ms", lambda: plan.beta_forward_shifted(out, 1, 4)),
                     ("shifted_depth2_block16_ms", lambda: plan.beta_forward_shifted(out, 2, 16)),
                     ("shifted_depth2_block4_ms", lambda: plan.beta_forward_shifted(out, 2, 4))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(max(3, steps // 5)):
            fn()
        e1.record()
        torch.cuda.synchronize()
        res[name] = round(e0.elapsed_time(e1) / max(3, steps // 5), 4)
    C = B * (B + 1) * (2 * B + 1) // 6
    flops = shifted_depth1_flops(B, batch)
    for form in ("depth1", "depth2_block16"):
        ach = flops / (res[f"shifted_{form}_ms"] * 1e-3)
        res[f"roofline_{form}"] = {"bound": "mfma", "achieved": round(ach / 1e12, 3),
                                   "peak": MFMA_PEAK["c128"] / 1e12, "unit": "TFLOP/s",
                                   "frac": round(ach / MFMA_PEAK["c128"], 4)}
    plan.close()
    return res


def mixed_batch(steps: int, warmup: int, untuned: bool):
    """The mixed-bandlimit step: 256 signals at B = 32 plus 64 with B from
    {16, 24, 32, 48, 64}, FP32, one plan (autotuned; untuned: also with the
    autotuner off)."""
    import numpy as np
    import torch

    import paper_2605_23923_amd as su2
    import synth

    out = {}
    Bs = [32] * 256 + synth.bandlimits_mixed(64, seed=33)
    ns = sum((2 * b) ** 3 for b in Bs)
    nc = sum(b * (b + 1) * (2 * b + 1) // 6 for b in Bs)
    rng = np.random.default_rng(3)
    x = torch.from_numpy((rng.uniform(-1, 1, ns) + 1j * rng.uniform(-1, 1, ns)).astype(np.complex64)).to("cuda")
    c = torch.from_numpy(((rng.standard_normal(nc) + 1j * rng.standard_normal(nc)) / np.sqrt(2)).astype(np.complex64)).to("cuda")
    out["mixed_320_signals_c64"] = run_whole(lambda: su2.MixedPlan(Bs, "c64"), x, c, steps, warmup, len(Bs))
    out["mixed_320_signals_c64"]["signals"] = "256 x B=32 + 64 x B in {16,24,32,48,64} (seed 33)"
    counts = {b: Bs.count(b) for b in sorted(set(Bs))}
    out["mixed_320_signals_c64"]["step_hbm_frac"] = step_hbm_frac(counts, "c64",
                                                                  out["mixed_320_signals_c64"]["ms_per_step"])
    if untuned:
        # the same step with the autotuner off (default tile shapes, 2 workgroups per CU)
        prev = os.environ.get("SU2_AUTOTUNE")
        os.environ["SU2_AUTOTUNE"] = "0"
        try:
            out["mixed_320_signals_c64_untuned"] = run_whole(lambda: su2.MixedPlan(Bs, "c64"), x, c, steps, warmup,
                                                             len(Bs))
        finally:
            if prev is None:
                del os.environ["SU2_AUTOTUNE"]
            else:
                os.environ["SU2_AUTOTUNE"] = prev
    del x, c
    torch.cuda.empty_cache()
    return out


def secondary_configs(steps: int, warmup: int):
    """The other workload shapes, timed through the public calls."""
    import numpy as np
    import torch

    import paper_2605_23923_amd as su2
    import synth

    out = mixed_batch(steps, warmup, untuned=True)
    out["b64_batch32_beta_forward_shifted_c64"] = shifted_forms(steps)
    # one signal at B = 64 (the table, read once per launch, then outweighs the
    # ring spectra), forward and inverse timed separately, FP32 and FP64
    for dt, npdt in (("c64", np.complex64), ("c128", np.complex128)):
        x = torch.from_numpy(synth.samples_uniform(64, 1, seed=2, dtype=npdt)).to("cuda")
        c = torch.from_numpy(synth.coeffs(64, 1, seed=2, spectrum="decay", dtype=npdt)).to("cuda")
        out[f"b64_batch1_{dt}"] = run_separate(lambda: su2.Plan(64, 1, dt), x, c, steps, warmup)
        del x, c
    torch.cuda.empty_cache()
    # B = 128, batch 16, split-BF16 contraction
    B, batch = 128, 16
    N = 2 * B
    x = torch.from_numpy(synth.samples_uniform(B, batch, seed=4, dtype=np.complex64)).to("cuda")
    c = torch.from_numpy(synth.coeffs(B, batch, seed=4, dtype=np.complex64)).to("cuda")
    out["b128_batch16_c64_bf16x3"] = run_whole(lambda: su2.Plan(B, batch, "c64_bf16x3"), x, c, max(2, steps // 5),
                                               1, batch)
    out["b128_batch16_c64_tables_on_the_fly"] = run_whole(lambda: su2.Plan(B, batch, "c64", tables="on_the_fly"),
                                                         x, c, max(2, steps // 5), 1, batch)
    # the same shape with the plain FP32 contraction (stored table), beside the split-BF16 one
    out["b128_batch16_c64"] = run_whole(lambda: su2.Plan(B, batch, "c64"), x, c, max(2, steps // 5), 1, batch)
    for key, m in (("b128_batch16_c64_bf16x3", "c64_bf16x3"), ("b128_batch16_c64", "c64")):
        out[key]["step_hbm_frac"] = step_hbm_frac({B: batch}, m, out[key]["ms_per_step"])
    del x, c
    torch.cuda.empty_cache()
    # and in FP64 throughout
    x = torch.from_numpy(synth.samples_uniform(B, batch, seed=4, dtype=np.complex128)).to("cuda")
    c = torch.from_numpy(synth.coeffs(B, batch, seed=4, dtype=np.complex128)).to("cuda")
    out["b128_batch16_c128"] = run_whole(lambda: su2.Plan(B, batch, "c128"), x, c, max(2, steps // 5), 1, batch)
    out["b128_batch16_c128"]["step_hbm_frac"] = step_hbm_frac({B: batch}, "c128", out["b128_batch16_c128"]["ms_per_step"])
    del x, c
    torch.cuda.empty_cache()
    return out


def measured_peaks():
    """What this device sustains, from the library's calibration kernels
    (su2fft_calib.h): a streaming copy and fill of 1 GiB buffers (HBM) and
    back-to-back 16x16 matrix-core products at 8 workgroups of 4 waves per CU,
    each the fastest of 5 timed launches (HIP events on the launch stream)."""
    import torch

    import paper_2605_23923_amd as su2

    def best_ms(fn, reps=5):
        fn()
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        return min(times)

    nbytes = 1 << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    su2.calib_fill(src, 1.0)
    copy_ms = best_ms(lambda: su2.calib_copy(src, dst))
    fill_ms = best_ms(lambda: su2.calib_fill(dst, 2.0))
    del src, dst
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    wg = 8 * cus
    out = torch.empty(wg * 256, dtype=torch.float32, device="cuda")
    mfma = {}
    for kind, iters in (("fp64", 400), ("fp32", 800), ("bf16", 1500)):
        flops = []
        ms = best_ms(lambda: flops.append(su2.calib_mfma(kind, wg, iters, out)))
        mfma[kind] = round(flops[-1] / (ms * 1e-3) / 1e12, 2)
    torch.cuda.synchronize()
    return {"copy_GBps": round(2 * nbytes / (copy_ms * 1e-3) / 1e9, 1),
            "fill_GBps": round(nbytes / (fill_ms * 1e-3) / 1e9, 1),
            "mfma_TFLOPs": mfma,
            "published": {"hbm_GBps": HBM_PEAK / 1e9,
                          "mfma_TFLOPs": {"fp64": MFMA_PEAK["c128"] / 1e12, "fp32": MFMA_PEAK["c64"] / 1e12,
                                          "bf16": MFMA_PEAK["c64_bf16x3"] / 1e12}},
            "method": "su2_calib_copy / su2_calib_fill over 1 GiB (copy counts read + write), su2_calib_mfma "
                      "16x16x4 FP64/FP32 and 16x16x32 BF16 at %d workgroups x 256 threads; best of 5" % wg}


def cpu_baseline(B: int, budget_s: float, threads: int = 0):
    """The oracle's direct sum on a bounded sample: the forward transform of one
    signal restricted to a subset of its coefficients (a few of every 2l), timed
    on the host (all cores, or `threads` of them); scaled to whole-signal
    transforms per second."""
    import numpy as np

    import oracle
    import synth

    if threads:
        all_threads = oracle.num_threads()
        oracle.set_num_threads(threads)
        try:
            return cpu_baseline(B, budget_s)
        finally:
            oracle.set_num_threads(all_threads)

    C = B * (B + 1) * (2 * B + 1) // 6
    x = synth.samples_uniform(B, 1, seed=5)[0]
    rng = np.random.default_rng(0)
    probe = rng.choice(C, 32, replace=False)
    t0 = time.perf_counter()
    oracle.forward(B, x, probe)
    per = (time.perf_counter() - t0) / probe.size
    count = int(min(C, max(64, budget_s / max(per, 1e-9))))
    sel = rng.choice(C, count, replace=False)
    t0 = time.perf_counter()
    oracle.forward(B, x, sel)
    dt = time.perf_counter() - t0
    return {"value": round(count / dt / C, 6), "unit": "transforms/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"forward, B={B}, 1 signal, {count} of {C} coefficients (direct quadrature sum, "
                      f"{(2 * B) ** 3} terms each), {dt:.1f} s; scaled by {C}/{count}"}


def cpu_fft_baselines(B: int):
    """A plain CPU FFT-based separated transform (scipy.fft + numpy matmul,
    all host cores), in float64 and in float32: forward and inverse
    transforms of a batch of 4 signals, best of 3 after a warm-up; tables
    built once per precision, before timing.  Returns the entries, the
    float64 forward first."""
    import numpy as np

    import oracle.cpu_fft as cf
    import synth

    x = synth.samples_uniform(B, 4, seed=5)
    c = synth.coeffs(B, 4, seed=6)
    out = []
    for dt, name in ((np.complex128, "float64"), (np.complex64, "float32")):
        plan = cf.CpuFFTPlan(B, dtype=dt)
        xd, cd = x.astype(dt), c.astype(dt)
        for direction, fn, arg in (("forward", plan.forward, xd), ("inverse", plan.inverse, cd)):
            fn(arg)
            best = 1e30
            for _ in range(3):
                t0 = time.perf_counter()
                fn(arg)
                best = min(best, time.perf_counter() - t0)
            out.append({"value": round(4 / best, 3), "unit": "transforms/s", "cores": plan.workers,
                        "kind": "cpu_fft",
                        "sample": f"{direction}, B={B}, batch 4, scipy.fft (workers={plan.workers}) + numpy matmul "
                                  f"in {name}, best of 3: {best:.2f} s; table build excluded"})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", default="c64", choices=["c128", "c64", "c64_bf16x3"],
                    help="precision mode of the headline number")
    ap.add_argument("--other-modes", default="c128,c64_bf16x3,c64_otf,c64_real,c64_so3",
                    help="comma-separated modes also timed and reported under 'modes' ('' for none); "
                         "'_otf' = Wigner-d values generated inside the contraction kernels, "
                         "'_real' = real-signal plan, '_so3' = SO(3) plan (integer degrees)")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-calibration", action="store_true",
                    help="skip the copy / fill / matrix-core calibration reported under 'measured_peaks'")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the mixed-bandlimit and B=128 workloads reported under 'other_workloads'")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a plain device-to-device copy of MB megabytes three times (reference for "
                         "the HBM byte counters) and exit")
    ap.add_argument("--workload", default="b64_batch32", choices=sorted(WORKLOADS),
                    help="b64_batch32 (default): the headline line.  b128_batch16: only the B=128 batch 16 shape "
                         "(256^3 grid), stage by stage for --mode and --other-modes, printed as one JSON object "
                         "(for profiling; not the headline line).  mixed_320: only the mixed-bandlimit step "
                         "(256 x B=32 + 64 x B in {16,24,32,48,64}, c64, autotuned), for profiling")
    ap.add_argument("--shifted-forms", action="store_true",
                    help="only time the forward contraction in its table and shifted-recurrence forms at B=64 "
                         "batch 32 (c64 plan), print that JSON object and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (got --gpus {args.gpus}); signals are independent, so a "
              "multi-GPU run would shard the batch by signal with no communication.", file=sys.stderr)
        sys.exit(2)

    if args.shifted_forms:
        print(json.dumps(shifted_forms(args.steps)))
        return

    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "repeats": 3}))
        return

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)

    B, batch = WORKLOADS[args.workload]
    digest = source_digest()
    import paper_2605_23923_amd as su2
    su2.Plan(4, 1, "c64").close()   # loads the code objects, so that plan_ms is set-up alone
    if args.workload == "mixed_320":
        res = mixed_batch(args.steps, args.warmup, untuned=False)
        print(json.dumps({"workload": args.workload, "steps": args.steps, **res, "source_digest": digest}), flush=True)
        return
    if args.workload != "b64_batch32":
        modes = {}
        for m in [args.mode] + [m for m in args.other_modes.split(",") if m and m != args.mode]:
            modes[m] = run_mode(m, B, batch, args.steps, args.warmup, False)
            print(f"bench.py: {args.workload} {m} done", file=sys.stderr, flush=True)
        print(json.dumps({"workload": args.workload, "B": B, "batch": batch, "steps": args.steps,
                          "modes": {m: {k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()}
                                    for m, r in modes.items()},
                          "source_digest": digest}), flush=True)
        return
    head = run_mode(args.mode, B, batch, args.steps, args.warmup, True)
    modes = {args.mode: head}
    for m in [m for m in args.other_modes.split(",") if m and m != args.mode]:
        modes[m] = run_mode(m, B, batch, max(5, args.steps // 2), args.warmup, False)

    dom = max(STAGES, key=lambda s: head["stage_ms"][s])
    dom_ms = head["stage_ms"][dom]
    ab = algorithmic_bytes(dom, B, batch, args.mode)
    achieved = ab / (dom_ms * 1e-3)
    roof = {"bound": "hbm", "kernel": kernel_name(dom, args.mode), "stage": dom, "achieved": round(achieved / 1e9, 2),
            "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": round(achieved / HBM_PEAK, 4),
            "algorithmic_bytes_per_launch": ab, "avg_launch_ms": round(dom_ms, 5),
            "traffic": measured_traffic(kernel_name(dom, args.mode), args.mode, digest)}

    line = {
        "metric": "SU(2) FFT transforms/s at B=64 batch 32; %HBM/MFMA peak; plain vs BF16x2",
        "value": round(head["transforms_per_s"], 2),
        "unit": "transforms/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE_NAME[base_mode(args.mode)], "data": "synthetic",
        "config": {"workload": "SU(2) transform chain (forward + inverse + adjoint), B=64 (2l<64), "
                               "128^3 Euler grid, batch 32, bandlimited Gaussian coefficients var (2l+1)^-2",
                   "B": B, "batch": batch, "grid": "128x128x128", "mode": args.mode,
                   "transforms_per_step": 3 * batch},
        "roofline": roof,
        "modes": {m: {k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()} for m, r in modes.items()},
        "source_digest": digest,
    }
    if not args.no_calibration:
        peaks = measured_peaks()
        line["measured_peaks"] = peaks
        roof["frac_of_measured_copy"] = round(achieved / (peaks["copy_GBps"] * 1e9), 4)
    if not args.no_secondary:
        line["other_workloads"] = secondary_configs(max(5, args.steps // 2), args.warmup)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(B, args.cpu_budget)
        line["cpu_baseline_1core"] = cpu_baseline(B, args.cpu_budget / 3, threads=1)
        fft = cpu_fft_baselines(B)
        line["cpu_fft_baseline"] = fft[0]
        line["cpu_fft_baselines"] = fft
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
