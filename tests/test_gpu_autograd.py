"""Autograd: the forward transform as a torch.autograd.Function whose backward
is the adjoint kernel chain (for a C-linear map F, PyTorch's complex convention
gives grad_x = F^H grad_y).

Loss (the differentiation configuration): L = sum_b sum_l (2l+1) ||fhat_b(l) - T_b(l)||_F^2.
Central differences with h = 1e-3 evaluated in FP64 are exact for this
quadratic loss up to rounding, so they pin the gradient directly:
  (L(x + h v) - L(x - h v)) / (2 h) = Re <grad, v>.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_23923_amd as su2
import synth

pytestmark = pytest.mark.gpu


def _weights(B, device, dtype):
    tl = synth.two_l_of_index(B)
    return torch.from_numpy((tl + 1).astype(np.float64)).to(device=device, dtype=dtype)


def _loss(fhat, target, w):
    return (w * (fhat - target).abs() ** 2).sum()


def _fd_directional(plan64, x, v, target, w, h=1e-3):
    with torch.no_grad():
        lp = _loss(plan64.forward((x + h * v).contiguous()), target, w)
        lm = _loss(plan64.forward((x - h * v).contiguous()), target, w)
    return ((lp - lm) / (2 * h)).item()


def test_autograd_fp64_matches_central_differences():
    B, batch = 8, 2
    plan = su2.Plan(B, batch, "c128")
    x = torch.from_numpy(synth.samples_uniform(B, batch, seed=5)).to("cuda").requires_grad_(True)
    target = torch.from_numpy(synth.coeffs(B, batch, seed=55)).to("cuda")
    w = _weights(B, "cuda", torch.float64)
    loss = _loss(su2.SU2Transform.apply(x, plan), target, w)
    loss.backward()
    g = x.grad.detach()
    rng = np.random.default_rng(1)
    xd = x.detach()
    for i in range(8):
        v = torch.from_numpy(rng.standard_normal(xd.shape) + 1j * rng.standard_normal(xd.shape)).to("cuda")
        v = v / v.abs().pow(2).sum().sqrt()
        fd = _fd_directional(plan, xd, v, target, w)
        an = (g.conj() * v).real.sum().item()
        assert abs(fd - an) <= 1e-9 * max(1.0, abs(fd)), (i, fd, an)
    flat = xd.reshape(-1)
    for idx in rng.choice(flat.numel(), 16, replace=False):
        for unit in (1.0, 1j):
            v = torch.zeros_like(flat)
            v[idx] = unit
            fd = _fd_directional(plan, xd, v.reshape(xd.shape), target, w)
            an = (g.reshape(-1)[idx].conj() * unit).real.item()
            assert abs(fd - an) <= 1e-9 * max(1.0, abs(fd)), (idx, unit, fd, an)


def test_gradcheck_tiny():
    B = 2
    plan = su2.Plan(B, 1, "c128")
    x = torch.from_numpy(synth.samples_uniform(B, 1, seed=7)).to("cuda").requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: su2.SU2Transform.apply(t, plan), (x,), eps=1e-6, atol=1e-8)


def test_config5_b64_batch32_fp32_gradient():
    """B = 64, batch 32, FP32 samples uniform on [-1, 1]: the gradient of the FP32
    autograd path against (a) central differences of the FP64 loss along random
    directions and (b) the oracle's adjoint of 2 (2l+1)(fhat - T), with fhat from
    the oracle's direct forward of signal 0, at sampled sample points."""
    B, batch = 64, 32
    plan32 = su2.Plan(B, batch, "c64")
    plan64 = su2.Plan(B, batch, "c128")
    xh = synth.samples_uniform(B, batch, seed=5, dtype=np.complex64)
    th = synth.coeffs(B, batch, seed=55)
    x = torch.from_numpy(xh).to("cuda").requires_grad_(True)
    target32 = torch.from_numpy(th.astype(np.complex64)).to("cuda")
    w32 = _weights(B, "cuda", torch.float32)
    loss = _loss(su2.SU2Transform.apply(x, plan32), target32, w32)
    loss.backward()
    g = x.grad.detach().to(torch.complex128)
    # (a) directional central differences in FP64
    x64 = torch.from_numpy(xh.astype(np.complex128)).to("cuda")
    target64 = torch.from_numpy(th).to("cuda")
    w64 = _weights(B, "cuda", torch.float64)
    # An FP32 gradient carries an error of a few 1e-6 of its norm in every
    # direction, so Re <grad, v> is checked against |grad| |v| (Cauchy-Schwarz
    # scale), plus the rounding of the FP64 loss differences (eps |L| / h).
    # One direction is the FP32 gradient itself, so the projection is large.
    rng = np.random.default_rng(2)
    gnorm = g.abs().pow(2).sum().sqrt().item()
    with torch.no_grad():
        L64 = _loss(plan64.forward(x64), target64, w64).item()
    dirs = [g / gnorm]
    for i in range(3):
        v = torch.from_numpy(rng.standard_normal(xh.shape) + 1j * rng.standard_normal(xh.shape)).to("cuda")
        dirs.append(v / v.abs().pow(2).sum().sqrt())
    for i, v in enumerate(dirs):
        fd = _fd_directional(plan64, x64, v, target64, w64)
        an = (g.conj() * v).real.sum().item()
        err = abs(fd - an)
        bound = 1e-5 * gnorm + 1e-15 * abs(L64) / 1e-3
        print(f"direction {i}: fd {fd:.10e} autograd {an:.10e} |diff| {err:.2e} "
              f"(|grad| {gnorm:.3e}, bound {bound:.2e})", flush=True)
        assert err <= bound
    # (b) oracle adjoint at sampled points of signal 0
    C = oracle.num_coeffs(B)
    x0 = xh[0].astype(np.complex128)
    fhat0 = oracle.forward(B, x0)
    gcoef = 2.0 * (synth.two_l_of_index(B) + 1) * (fhat0 - th[0])
    N = 2 * B
    pts = rng.choice(N ** 3, 48, replace=False)
    ref = oracle.adjoint(B, gcoef, pts)
    got = g[0].reshape(-1).cpu().numpy()[pts]
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"gradient vs oracle adjoint (48 points): rel {rel:.2e}")
    assert rel <= 2e-5
    assert C == fhat0.size
