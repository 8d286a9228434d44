"""fht_forward_noalloc (the forward for callers that cannot allocate) against
fht_forward, through the C ABI.

Both run the same kernels in the same order, so outputs must agree bit for
bit, integer and float alike; two calls in a row share one device scratch,
the second on a smaller image, so a stale scratch would show.  The 61 x 47
call is also checked against the oracle.
"""
import numpy as np
import pytest

import workloads as WL
from oracle import fht_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_07351_amd as F
    return F


def _both(F, img_np, split="S"):
    """Outputs of fht_forward and of fht_forward_noalloc for one image."""
    img = torch.from_numpy(np.ascontiguousarray(img_np)).cuda()
    plan = F.Plan(img.shape[0], img.shape[1], img.dtype, split)
    F.fht_plan_upload(plan.handle)
    ref = plan.new_out()
    ws = plan.new_ws()
    stream = torch.cuda.current_stream().cuda_stream
    F.fht_forward(plan.handle, img.data_ptr(), ref.data_ptr(), ws.data_ptr(), stream)
    got = torch.full_like(ref, -7)
    F.fht_forward_noalloc(plan.handle, img.data_ptr(), got.data_ptr(), stream)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy(), plan


@pytest.mark.parametrize("split", ["S", "T"])
def test_noalloc_equals_forward_two_calls_u8(F, split):
    rng = WL.rng_for(2, salt=31)
    for R, C in [(1021, 1021), (517, 300)]:
        ref, got, plan = _both(F, WL.edge_map(rng, R, C), split)
        assert plan.ws_bytes <= F.NOALLOC_WS_BYTES
        assert (got == ref).all(), (R, C, int((got != ref).sum()))


def test_noalloc_equals_forward_two_calls_f32(F):
    rng = WL.rng_for(4, salt=31)
    for R, C in [(384, 257), (129, 70)]:
        ref, got, _ = _both(F, WL.normal_f32(rng, R, C))
        assert np.array_equal(got, ref), (R, C)


def test_noalloc_matches_oracle_61x47(F):
    img = WL.uniform_u8(WL.rng_for(1), 61, 47)
    _, got, plan = _both(F, img)
    ref = O.hough4(img, 0)
    for q in range(4):
        o = plan.shapes[q]
        off = F.fht_plan_out_offset(plan.handle, q)
        assert (got[off:off + o[0] * o[1]].reshape(o) == ref[q]).all(), q


def test_noalloc_rejects_without_launching(F):
    # a workspace above the scratch: rejected on the host
    big = F.Plan(2048, 2048, torch.uint8, "S")
    assert big.ws_bytes > F.NOALLOC_WS_BYTES
    F.fht_plan_upload(big.handle)
    img = torch.zeros(2048, 2048, dtype=torch.uint8, device="cuda")
    out = big.new_out()
    with pytest.raises(F.FhtError, match="FHT_EINVAL"):
        F.fht_forward_noalloc(big.handle, img.data_ptr(), out.data_ptr(), None)
    # tables not on the device yet: rejected (uploading would allocate)
    fresh = F.Plan(33, 35, torch.uint8, "S")
    img = torch.zeros(33, 35, dtype=torch.uint8, device="cuda")
    out = fresh.new_out()
    with pytest.raises(F.FhtError, match="FHT_EINVAL"):
        F.fht_forward_noalloc(fresh.handle, img.data_ptr(), out.data_ptr(), None)
    torch.cuda.synchronize()
