"""Backward pass of the soft-alignment loss L = sum_a g[a] lse_img[a]
(align_pairs_backward and the RadialAlignLSE autograd function).

* Small problems (the FD subset of the differentiation workload, and a
  non-Hermitian one): the GPU gradients against the FP64 oracle gradient,
  which is itself pinned to central differences (test_oracle_pins).
* Differentiation workload (2048 noisy images x 256 templates, Q=256, T=9,
  H=16): the FP32 plan's gradients against the FP64 plan's on the same inputs
  and U, and central differences of the library's own FP64 landscape on a
  subset of it.

Bar: max |g - g_ref| <= 1e-6 max |g_ref| (and of the directional derivative
for the finite-difference checks).  The backward arithmetic is FP64 and
recomputes the log-sum-exp normalisation itself; what limits FP32 plans is
their FP32 ring operands (~1e-7 relative).  FP64 plans agree with the oracle
to rounding (the oracle is given the same f32-rounded inv_sigma2 and g).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2202_07235_amd as rs
import synth
from tests._parity import host_inputs, to_device

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _rel(x, ref):
    return float(np.abs(np.asarray(x) - np.asarray(ref)).max() / np.abs(np.asarray(ref)).max())


def _small(cfg, seed, precision):
    P = synth.make_problem(cfg, seed=seed)
    A, B = to_device(P, precision)
    A_h, B_h = host_inputs(A, B)
    U, _ = oracle.principal_vectors(oracle.kernel_C(B_h, P.w, cfg.Q))
    X = oracle.landscape(A_h, B_h, U, cfg.H, P.k, P.w, P.delta)
    s = float(np.float32(3.0 / np.abs(X).max()))   # the library takes inv_sigma2 as f32
    g = np.random.default_rng(seed).standard_normal(cfg.n_img).astype(np.float32).astype(np.float64)
    return P, A, B, A_h, B_h, U, s, g


CASES = [("fp32", True), ("bf16x3", True), ("fp64", True), ("fp64", False)]


@pytest.mark.parametrize("precision,hermitian", CASES)
def test_backward_matches_oracle_gradient(precision, hermitian):
    if hermitian:
        cfg = synth.config("diff_fd")
    else:   # complex (non-conjugate-symmetric) inputs: full spectrum in the library
        cfg = synth.config("tiny", n_img=6, n_tgt=5, T=9, H=8)
    P, A, B, A_h, B_h, U, s, g = _small(cfg, 71 + len(precision), precision)
    gB_or, gU_or = oracle.lse_grad(A_h, B_h, U, cfg.H, P.k, P.w, P.delta, s, g)
    UH = torch.tensor(np.ascontiguousarray(U[:, :cfg.H]))
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision=precision, hermitian=hermitian, products=6, U=UH)
    o = plan.pairs("lse", inv_sigma2=s)
    gB, gU = plan.backward(s, o["lse_img"], torch.tensor(g, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    eB = _rel(gB.cpu().to(torch.complex128).numpy(), gB_or)
    eU = _rel(gU.cpu().numpy(), gU_or)
    print(f"{precision} hermitian={hermitian}: dL/dB rel err {eB:.2e}, dL/dU rel err {eU:.2e}")
    assert eB <= TOL and eU <= TOL


@pytest.mark.parametrize("precision,H,Q", [("fp32", 24, 64), ("fp64", 32, 64), ("fp32", 16, 128), ("fp64", 16, 256),
                                           ("fp32", 16, 512)])
def test_backward_more_shapes_match_oracle_gradient(precision, H, Q):
    """Ranks above 16 take the contraction kernels' wider rank blocking (eight
    ranks per thread, two rank values per thread and image tile); Q = 128 and
    256 give the P-hat step a last pass over frequencies holding only Q/2, and
    Q = 512 is the largest angle count of its wave-per-row kernel; 5 targets x
    9 translations leave a partial last tile of columns."""
    cfg = synth.config("diff_fd", K=32, H=H, n_tgt=5, Q=Q)
    P, A, B, A_h, B_h, U, s, g = _small(cfg, 90 + H + Q, precision)
    gB_or, gU_or = oracle.lse_grad(A_h, B_h, U, cfg.H, P.k, P.w, P.delta, s, g)
    UH = torch.tensor(np.ascontiguousarray(U[:, :cfg.H]))
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision=precision, hermitian=True, U=UH)
    o = plan.pairs("lse", inv_sigma2=s)
    gB, gU = plan.backward(s, o["lse_img"], torch.tensor(g, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    eB = _rel(gB.cpu().to(torch.complex128).numpy(), gB_or)
    eU = _rel(gU.cpu().numpy(), gU_or)
    print(f"{precision} H={H} Q={Q}: dL/dB rel err {eB:.2e}, dL/dU rel err {eU:.2e}")
    assert eB <= TOL and eU <= TOL


def test_backward_outputs_are_optional_and_consistent():
    cfg = synth.config("diff_fd")
    P, A, B, A_h, B_h, U, s, g = _small(cfg, 5, "fp32")
    UH = torch.tensor(np.ascontiguousarray(U[:, :cfg.H]))
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision="fp32", U=UH)
    o = plan.pairs("lse", inv_sigma2=s)
    gt = torch.tensor(g, dtype=torch.float32, device="cuda")
    gB, gU = plan.backward(s, o["lse_img"], gt)
    gB_only, none_U = plan.backward(s, o["lse_img"], gt, want_U=False)
    none_B, gU_only = plan.backward(s, o["lse_img"], gt, want_B=False)
    assert none_U is None and none_B is None
    assert torch.equal(gB, gB_only) and torch.equal(gU, gU_only)


def test_autograd_function_matches_oracle():
    cfg = synth.config("diff_fd")
    P, A, B, A_h, B_h, U, s, g = _small(cfg, 9, "fp32")
    Bv = B.clone().requires_grad_(True)
    Ut = torch.tensor(np.ascontiguousarray(U[:, :cfg.H]), device="cuda", requires_grad=True)
    lse = rs.RadialAlignLSE.apply(A, Bv, Ut, P.k, P.w, P.delta, s, "fp32", True)
    (lse * torch.tensor(g, dtype=torch.float32, device="cuda")).sum().backward()
    gB_or, gU_or = oracle.lse_grad(A_h, B_h, U, cfg.H, P.k, P.w, P.delta, s, g)
    _, li = oracle.lse(oracle.landscape(A_h, B_h, U, cfg.H, P.k, P.w, P.delta), s)
    assert np.abs(lse.detach().cpu().numpy() - li).max() <= 1e-5 * np.abs(li).max()
    assert _rel(Bv.grad.cpu().to(torch.complex128).numpy(), gB_or) <= TOL
    assert _rel(Ut.grad.cpu().numpy(), gU_or) <= TOL


def _loss64(A, B, U, P, H, s, g):
    """FP64 loss from the library's FP64 full-spectrum landscape (FULL output),
    reduced in FP64.  The full-spectrum path treats every polar sample as free,
    as the gradient does, so the perturbation need not be conjugate-symmetric."""
    plan = rs.Plan(A, B, P.k, P.w, P.delta, H, precision="fp64", hermitian=False, U=U)
    X = plan.pairs("full")["X"].real
    lp = torch.logsumexp((s * X).flatten(2), dim=2)
    return float((g * torch.logsumexp(lp, dim=1)).sum())


def test_diff_workload_fp32_backward_matches_fp64_and_finite_differences():
    cfg = synth.config("diff")
    P = synth.make_problem(cfg, seed=5005, device="cuda")
    A32 = P.A.to(torch.complex64).contiguous()
    B32 = P.B.to(torch.complex64).contiguous()
    P.A = P.B = None
    A64, B64 = A32.to(torch.complex128), B32.to(torch.complex128)
    U = rs.Plan(A32, B32, P.k, P.w, P.delta, cfg.H, precision="fp32").U_lambda()[0][:, :cfg.H].contiguous()
    s = 1.0   # sigma^2 = 1
    g = torch.ones(cfg.n_img, dtype=torch.float32, device="cuda")
    grads = {}
    for prec, A, B in (("fp32", A32, B32), ("fp64", A64, B64)):
        plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision=prec, U=U)
        o = plan.pairs("lse", inv_sigma2=s)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        gB, gU = plan.backward(s, o["lse_img"], g)
        e1.record()
        torch.cuda.synchronize()
        print(f"diff workload backward ({prec} plan): {e0.elapsed_time(e1):.1f} ms")
        grads[prec] = (gB.to(torch.complex128).cpu().numpy(), gU.cpu().numpy())
        del plan
    eB = _rel(grads["fp32"][0], grads["fp64"][0])
    eU = _rel(grads["fp32"][1], grads["fp64"][1])
    print(f"diff workload: FP32 vs FP64 plan gradients: dL/dB {eB:.2e}, dL/dU {eU:.2e}")
    assert eB <= TOL and eU <= TOL

    # central differences of the FP64 landscape on a subset (128 images x 32 templates)
    na, nb = 128, 32
    A, B = A64[:na].contiguous(), B64[:nb].contiguous()
    gs = torch.ones(na, dtype=torch.float64, device="cuda")
    plan = rs.Plan(A, B, P.k, P.w, P.delta, cfg.H, precision="fp64", U=U)
    o = plan.pairs("lse", inv_sigma2=s)
    gB, gU = plan.backward(s, o["lse_img"], gs.to(torch.float32))
    gen = torch.Generator(device="cuda").manual_seed(3)
    V = torch.randn(B.shape, dtype=torch.complex128, device="cuda", generator=gen)
    hB = 1e-6 * float(B.abs().max()) / float(V.abs().max())
    fd = (_loss64(A, B + hB * V, U, P, cfg.H, s, gs) - _loss64(A, B - hB * V, U, P, cfg.H, s, gs)) / (2 * hB)
    an = float((torch.conj(gB) * V).real.sum())
    print(f"directional derivative along B: FD {fd:.10e}, backward {an:.10e}")
    assert abs(fd - an) <= TOL * abs(an)
    W = torch.randn(U.shape, dtype=torch.float64, device="cuda", generator=gen)
    hU = 1e-6
    fdU = (_loss64(A, B, U + hU * W, P, cfg.H, s, gs) - _loss64(A, B, U - hU * W, P, cfg.H, s, gs)) / (2 * hU)
    anU = float((gU * W).sum())
    print(f"directional derivative along U: FD {fdU:.10e}, backward {anU:.10e}")
    assert abs(fdU - anU) <= TOL * abs(anU)
