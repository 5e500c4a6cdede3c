"""GPU: lalm_dot_f64_noalloc (no plan, no allocation: the library's static
per-GPU scratch) gives the bits of lalm_dot_f64 on the same inputs, on two
calls in a row, the second with a smaller input, and rejects sizes beyond
its stated maximum."""
import numpy as np
import pytest

from _helpers import ensure_built, say

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_noalloc_dot_equals_planned_dot():
    ensure_built()
    from paper_1402_4381_amd import lalm
    plan = lalm.lalm_plan_geometry(synth.geometry_of(synth.get_config("tiny2d")), 3)
    rng = np.random.default_rng(61)
    for n in (3_000_017, 70_001):              # the second call smaller than the first
        a = torch.as_tensor(rng.normal(size=n).astype(np.float32), device=DEV)
        b = torch.as_tensor(rng.normal(size=n).astype(np.float32), device=DEV)
        ref = torch.zeros(1, dtype=torch.float64, device=DEV)
        got = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
        lalm.lalm_dot_f64(plan, a, b, ref)
        lalm.lalm_dot_f64_noalloc(a, b, got)
        want = float(np.dot(a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)))
        say("n=%d noalloc %.17g planned %.17g fp64 %.17g" % (n, got.item(), ref.item(), want))
        assert torch.equal(got, ref)
        assert abs(got.item() - want) <= 1e-11 * float(np.sum(np.abs(a.cpu().numpy().astype(np.float64)
                                                                     * b.cpu().numpy().astype(np.float64))))
    z = torch.zeros(1, device=DEV)
    with pytest.raises(lalm.LalmError):
        lalm._check(lalm._lib.lalm_dot_f64_noalloc(lalm._dev(z, "a"), lalm._dev(z, "b"), (1 << 40) + 1,
                                                   lalm._dev(ref, "o", dtype="float64"), lalm._stream(None)))
