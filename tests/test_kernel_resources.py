"""The compiler's resource report for the library as built: no kernel keeps
values in scratch memory (private per-lane stack or register spills), which
costs a contraction kernel several times its run time."""
import json
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
REPORT = os.path.join(HERE, "..", "paper_2605_23923_amd", "kernel_resources.json")

# kernel (demangled, up to the argument list) -> largest scratch bytes per lane
# allowed; none at present
ALLOWED = {}


def _report():
    if not os.path.exists(REPORT):
        pytest.skip("library not built here (no kernel resource report)")
    with open(REPORT) as fh:
        return json.load(fh)


def test_report_covers_the_transform_kernels():
    names = " ".join(_report())
    for k in ("ring_forward_fast<float, 64, false>", "ring_inverse_fast<double, 128, false>",
              "beta_forward_kernel<float, 2, 4, 32>", "beta_inverse_kernel<double, 16, 16, 2>", "beta_inverse_kernel<double, 8, 16, 1>", "beta_forward_bf16x3_kernel<4>",
              "ring_cols_forward_large<float>", "beta_forward_otf_kernel<float, 2, 32>"):
        assert k in names, k


def test_no_kernel_uses_scratch():
    bad = []
    for name, r in _report().items():
        short = name.split("(")[0].replace("void ", "")
        limit = ALLOWED.get(short, 0)
        if r.get("scratch_bytes", 0) > limit or (limit == 0 and r.get("vgpr_spill", 0) > 0):
            bad.append((short, r.get("scratch_bytes"), r.get("vgpr_spill")))
    assert not bad, bad
