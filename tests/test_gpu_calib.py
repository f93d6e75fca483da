"""The calibration kernels behind bench.py's measured peaks: the copy and fill
move exactly the bytes they claim, and the matrix-core kernel computes the
products it is credited with (checked against numpy on the lane values the
kernel feeds: a = lane mod 3 + 1, b = lane mod 5 + 1)."""
import numpy as np
import pytest
import torch

import paper_2605_23923_amd as su2

pytestmark = pytest.mark.gpu

STEPS, CHAINS = 16, 4   # products per chain and loop trip, independent chains per wave


@pytest.mark.parametrize("nbytes", [16, 4096 + 48, (1 << 22) + 16 * 37])
def test_copy_and_fill_are_exact(nbytes):
    g = torch.Generator().manual_seed(nbytes)
    src = torch.randint(-2**31, 2**31 - 1, (nbytes // 4 + 8,), generator=g, dtype=torch.int32).to("cuda")
    dst = torch.zeros_like(src)
    su2.calib_copy(src[: nbytes // 4], dst[: nbytes // 4])
    torch.cuda.synchronize()
    assert torch.equal(dst[: nbytes // 4], src[: nbytes // 4])
    assert int(dst[nbytes // 4:].abs().sum()) == 0          # nothing past the end
    f = torch.zeros(nbytes // 4 + 8, dtype=torch.float32, device="cuda")
    su2.calib_fill(f[: nbytes // 4], 3.5)
    torch.cuda.synchronize()
    assert bool((f[: nbytes // 4] == 3.5).all()) and bool((f[nbytes // 4:] == 0).all())


def _expected(kind, workgroups, iters):
    lane = np.arange(64)
    a, b = (lane % 3 + 1).astype(np.float64), (lane % 5 + 1).astype(np.float64)
    per_k = 8.0 if kind == "bf16" else 1.0     # 16x16x32 BF16: 8 equal K values per lane
    # D[i][j] = sum over the 4 K groups of A[i][g] B[g][j] (lanes i + 16 g, j + 16 g)
    d = np.zeros((16, 16))
    for g in range(4):
        d += per_k * np.outer(a[16 * g:16 * g + 16], b[16 * g:16 * g + 16])
    # lane l holds rows 4 (l // 16) + e, e = 0..3, of column l % 16
    per_lane = np.array([sum(d[4 * (l // 16) + e, l % 16] for e in range(4)) for l in range(64)])
    per_lane *= CHAINS * STEPS * iters
    return np.tile(per_lane, workgroups * 4)


@pytest.mark.parametrize("kind", ["fp64", "fp32", "bf16"])
def test_mfma_kernel_computes_the_credited_products(kind):
    workgroups, iters = 3, 2
    out = torch.full((workgroups * 256,), -1.0, dtype=torch.float32, device="cuda")
    flops = su2.calib_mfma(kind, workgroups, iters, out)
    torch.cuda.synchronize()
    k = 32 if kind == "bf16" else 4
    assert flops == workgroups * 4 * iters * STEPS * CHAINS * 2 * 16 * 16 * k
    np.testing.assert_array_equal(out.cpu().numpy().astype(np.float64), _expected(kind, workgroups, iters))
