"""The adjoint (back-projection) kernels against the oracle, on the GPU.

fht_adjoint must equal the oracle's back-projection along the patterns
(``adjoint_lanes``/``adjoint4``) and the transpose of the oracle's explicit
operator matrix, and ``HoughFunction`` must pass an FP64 finite-difference
gradcheck.  Float64 is held to 1e-12 of the line scale, float32 to 1e-5 (the
scale of an image-gradient pixel is the back-projection of |G|).
"""
import numpy as np
import pytest
import torch

import paper_2411_07351_amd as F
from oracle import fht_oracle as O

pytestmark = pytest.mark.gpu

SIGMA = {0: 1, 1: -1, 2: 1, 3: -1}


def _gout(plan, Gs, dtype):
    g = torch.zeros(plan.out_elems, dtype=dtype)
    for q, G in Gs.items():
        off = plan.offsets[q]
        g[off:off + G.size] = torch.from_numpy(G.ravel()).to(dtype)
    return g.cuda()


def _run(plan, Gs, dtype):
    g = plan.adjoint(_gout(plan, Gs, dtype))
    torch.cuda.synchronize()
    return g.double().cpu().numpy()


@pytest.mark.parametrize("split", ["S", "T"])
@pytest.mark.parametrize("shape", [(13, 11), (11, 13), (7, 5), (16, 3), (1, 5), (5, 1), (1, 1),
                                   (61, 47), (100, 37), (17, 65)])
def test_adjoint_f64_equals_oracle(split, shape):
    R, C = shape
    plan = F.Plan(R, C, "f64", split)
    rng = np.random.default_rng(R * 100 + C)
    Gs = {q: rng.standard_normal(plan.shapes[q]) for q in range(4)}
    sp = 0 if split == "S" else 1
    ref = O.adjoint4(Gs, sp, shape)
    scale = O.adjoint4({q: np.abs(G) for q, G in Gs.items()}, sp, shape)
    got = _run(plan, Gs, torch.float64)
    assert np.all(np.abs(got - ref) <= 1e-12 * np.maximum(scale, 1.0))


@pytest.mark.parametrize("split", ["S", "T"])
@pytest.mark.parametrize("shape", [(13, 11), (11, 13), (7, 5), (16, 3)])
def test_adjoint_is_the_explicit_transpose(split, shape):
    R, C = shape
    plan = F.Plan(R, C, "f64", split)
    rng = np.random.default_rng(9)
    Gs = {q: rng.standard_normal(plan.shapes[q]) for q in range(4)}
    sp = 0 if split == "S" else 1
    ref = np.zeros(shape)
    for q, G in Gs.items():
        W, H = G.shape
        gA = (O.explicit_matrix(W, H, sp, SIGMA[q]).T @ G.ravel()).reshape(W, H)
        ref += gA if q < 2 else gA.T
    np.testing.assert_allclose(_run(plan, Gs, torch.float64), ref, rtol=0, atol=1e-12)


def test_adjoint_quadrant_subset():
    plan = F.Plan(19, 12, "f64", "S", quadrants=(1, 2))
    rng = np.random.default_rng(4)
    Gs = {q: rng.standard_normal(plan.shapes[q]) for q in (1, 2)}
    np.testing.assert_allclose(_run(plan, Gs, torch.float64), O.adjoint4(Gs, 0, (19, 12)),
                               rtol=0, atol=1e-12)


def test_adjoint_f32_384x257_within_tolerance():
    R, C = 384, 257
    plan = F.Plan(R, C, "f32", "S")
    rng = np.random.default_rng(2411_07351 + 4)
    Gs = {q: rng.standard_normal(plan.shapes[q]).astype(np.float32) for q in range(4)}
    ref = O.adjoint4(Gs, 0, (R, C))
    scale = O.adjoint4({q: np.abs(G) for q, G in Gs.items()}, 0, (R, C))
    got = _run(plan, Gs, torch.float32)
    assert np.all(np.abs(got - ref) <= 1e-5 * scale)


@pytest.mark.parametrize("split", ["S", "T"])
def test_dot_product_identity_at_full_size(split):
    # <F A, G> = <A, F^T G> holds at any size; checked in float64 on the GPU
    R, C = 384, 257
    plan = F.Plan(R, C, "f64", split)
    gen = torch.Generator(device="cuda").manual_seed(11)
    A = torch.randn(R, C, dtype=torch.float64, device="cuda", generator=gen)
    G = torch.randn(plan.out_elems, dtype=torch.float64, device="cuda", generator=gen)
    out = plan.new_out("cuda")
    plan.forward(A, out)
    lhs = float((out * G).sum())
    rhs = float((A * plan.adjoint(G)).sum())
    assert abs(lhs - rhs) <= 1e-10 * float((out.abs() * G.abs()).sum())


def test_gradcheck_f64_13x11():
    plan = F.Plan(13, 11, "f64", "S")
    img = torch.randn(13, 11, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: F.HoughFunction.apply(x, plan), (img,),
                                    eps=1e-6, atol=1e-7, rtol=1e-6)


def test_autograd_batch_of_float32_images():
    # config-4 shapes: gradients of a weighted sum of all quadrant outputs
    R, C, n = 384, 257, 4
    rng = np.random.default_rng(2411_07351 + 4)
    imgs = torch.from_numpy(rng.standard_normal((n, R, C)).astype(np.float32)).cuda()
    imgs.requires_grad_(True)
    plan = F.Plan(R, C, "f32", "S")
    wts = torch.from_numpy(rng.standard_normal((n, plan.out_elems)).astype(np.float32)).cuda()
    loss = sum((F.HoughFunction.apply(imgs[i], plan) * wts[i]).sum() for i in range(n))
    loss.backward()
    torch.cuda.synchronize()
    w = wts.double().cpu().numpy()
    for i in (0, n - 1):
        Gs = {q: w[i, plan.offsets[q]:plan.offsets[q] + R * C].reshape(plan.shapes[q])
              for q in range(4)}
        ref = O.adjoint4(Gs, 0, (R, C))
        scale = O.adjoint4({q: np.abs(G) for q, G in Gs.items()}, 0, (R, C))
        got = imgs.grad[i].double().cpu().numpy()
        assert np.all(np.abs(got - ref) <= 1e-5 * scale)


def test_uint8_adjoint_is_rejected():
    plan = F.Plan(9, 9, "u8", "S")
    g = torch.zeros(plan.out_elems, dtype=torch.int32, device="cuda")
    with pytest.raises(F.FhtError) as e:
        F.fht_adjoint(plan.handle, g.data_ptr(), g.data_ptr(), None, None)
    assert e.value.status == -2


def test_adjoint_many_equals_single_images():
    R, C, n = 61, 47, 5
    plan = F.Plan(R, C, "f64", "T")
    gen = torch.Generator(device="cuda").manual_seed(5)
    G = torch.randn(n, plan.out_elems, dtype=torch.float64, device="cuda", generator=gen)
    many = plan.adjoint_many(G)
    torch.cuda.synchronize()
    for b in range(n):
        assert torch.equal(many[b], plan.adjoint(G[b].contiguous())), b


def test_gradcheck_f64_batch_2x13x11():
    plan = F.Plan(13, 11, "f64", "S")
    img = torch.randn(2, 13, 11, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: F.HoughFunction.apply(x, plan), (img,),
                                    eps=1e-6, atol=1e-7, rtol=1e-6)


def test_autograd_batched_float32_384x257():
    # config-4 shapes through the batched forward and adjoint
    R, C, n = 384, 257, 3
    rng = np.random.default_rng(2411_07351 + 4)
    imgs = torch.from_numpy(rng.standard_normal((n, R, C)).astype(np.float32)).cuda()
    imgs.requires_grad_(True)
    quads = F.hough_autograd(imgs)
    wts = [torch.from_numpy(rng.standard_normal(tuple(q.shape)).astype(np.float32)).cuda()
           for q in quads]
    loss = sum((q * w).sum() for q, w in zip(quads, wts))
    loss.backward()
    torch.cuda.synchronize()
    for b in (0, n - 1):
        Gs = {q: wts[q][b].double().cpu().numpy() for q in range(4)}
        ref = O.adjoint4(Gs, 0, (R, C))
        scale = O.adjoint4({q: np.abs(G) for q, G in Gs.items()}, 0, (R, C))
        got = imgs.grad[b].double().cpu().numpy()
        assert np.all(np.abs(got - ref) <= 1e-5 * scale)
