"""The adjoint's gather steps (host tables) executed on the CPU.

``fht_plan_adjoint_tasks`` exposes the steps the adjoint kernels run; this
test executes them in NumPy with the kernels' semantics (mirror the output
gradient of negative-slope quadrants on the way in, gather level by level,
un-mirror, transpose column-lane views, sum) and compares the image gradient
with the oracle's direct back-projection along the patterns (Alg. 2), exactly
on integer-valued data.  No GPU is needed.
"""
import numpy as np
import pytest

import paper_2411_07351_amd as F
from oracle import fht_oracle as O


def _mirror(a):
    H = a.shape[1]
    return a[:, (-np.arange(H)) % H]


def interpret(plan, Gs, R, C):
    g = np.zeros((R, C))
    for q, G in Gs.items():
        tasks = F.fht_plan_adjoint_tasks(plan.handle, q >> 1)
        W, H = G.shape
        assert tasks.shape[1] == W
        cur = _mirror(G) if q & 1 else G.astype(np.float64)
        y = np.arange(H)
        for k in range(tasks.shape[0]):
            nxt = np.zeros((W, H))
            for x in range(W):
                p0, n, r0, right = (int(v) for v in tasks[k, x])
                assert n >= 1 and 0 <= p0 and p0 + n <= W
                for j in range(n):
                    shift = (r0 + j) if right else 0
                    nxt[x] += cur[p0 + j][(y - shift) % H]
            cur = nxt
        gA = _mirror(cur) if q & 1 else cur
        g += gA if q < 2 else gA.T
    return g


SHAPES = [(1, 1), (1, 7), (7, 1), (2, 2), (13, 11), (11, 13), (16, 3), (17, 5), (33, 7),
          (65, 4), (100, 37), (129, 5), (61, 47)]


@pytest.mark.parametrize("split", ["S", "T"])
@pytest.mark.parametrize("shape", SHAPES)
def test_adjoint_tasks_equal_oracle(split, shape):
    R, C = shape
    plan = F.Plan(R, C, "f64", split)
    rng = np.random.default_rng(R * 1000 + C)
    Gs = {q: rng.integers(-7, 8, size=plan.shapes[q]).astype(np.float64) for q in range(4)}
    ref = O.adjoint4(Gs, 0 if split == "S" else 1, (R, C))
    np.testing.assert_array_equal(interpret(plan, Gs, R, C), ref)


def test_adjoint_tasks_quadrant_subset():
    plan = F.Plan(19, 12, "f32", "S", quadrants=(1, 2))
    rng = np.random.default_rng(4)
    Gs = {q: rng.integers(-7, 8, size=plan.shapes[q]).astype(np.float64) for q in (1, 2)}
    np.testing.assert_array_equal(interpret(plan, Gs, 19, 12), O.adjoint4(Gs, 0, (19, 12)))


def test_split_t_fan_in_reaches_the_node_width():
    # Split_T gives a width-1 right child below w = 2^k + 1: all w parent rows
    # land on it, shifted by t
    plan = F.Plan(17, 5, "f32", "T")
    tasks = F.fht_plan_adjoint_tasks(plan.handle, 0)
    assert tasks[0, 16].tolist() == [0, 17, 0, 1]
    assert tasks[:, :, 1].max() == 17


def test_uint8_plans_have_no_adjoint():
    plan = F.Plan(9, 9, "u8", "S")
    with pytest.raises(F.FhtError) as e:
        F.fht_plan_adjoint_tasks(plan.handle, 0)
    assert e.value.status == -2
    assert F.fht_plan_adjoint_workspace_bytes(plan.handle) == 0


def interpret_fused(plan, Gs, R, C):
    """The gather launches fht_adjoint runs (fused passes), executed in NumPy."""
    g = np.zeros((R, C))
    for q, G in Gs.items():
        v = q >> 1
        W, H = G.shape
        cur = _mirror(G) if q & 1 else G.astype(np.float64)
        y = np.arange(H)
        levels = 0
        for p in range(F.fht_plan_adjoint_num_passes(plan.handle, v)):
            ps = F.fht_plan_adjoint_pass(plan.handle, v, p)
            offs, terms = ps["offs"], ps["terms"]
            levels += ps["levels"]
            assert offs.shape == (W + 1,) and offs[0] == 0 and offs[-1] == len(terms)
            assert (np.diff(offs) >= 1).all()
            assert ((terms[:, 0] >= 0) & (terms[:, 0] < W)).all()
            assert ((terms[:, 1] >= 0) & (terms[:, 1] < H)).all()
            nxt = np.zeros((W, H))
            for x in range(W):
                for row, sh in terms[offs[x]:offs[x + 1]]:
                    nxt[x] += cur[row][(y - sh) % H]
            cur = nxt
        assert levels == F.fht_plan_adjoint_tasks(plan.handle, v).shape[0]
        gA = _mirror(cur) if q & 1 else cur
        g += gA if q < 2 else gA.T
    return g


@pytest.mark.parametrize("split", ["S", "T"])
@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (7, 1), (13, 11), (16, 3), (17, 5), (33, 7),
                                   (100, 37), (129, 5), (61, 47)])
def test_fused_adjoint_passes_equal_oracle(split, shape):
    R, C = shape
    plan = F.Plan(R, C, "f64", split)
    rng = np.random.default_rng(R * 1000 + C + 7)
    Gs = {q: rng.integers(-7, 8, size=plan.shapes[q]).astype(np.float64) for q in range(4)}
    ref = O.adjoint4(Gs, 0 if split == "S" else 1, (R, C))
    np.testing.assert_array_equal(interpret_fused(plan, Gs, R, C), ref)
