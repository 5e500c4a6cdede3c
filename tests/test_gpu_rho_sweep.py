"""GPU check of the fixed-rho sweep on the 512x512 fan-beam workload (the
library's OS-LALM with continuation=False, rho_fixed = rho).  Sec. V orders
the methods by their RMS difference to x*: a smaller fixed rho accelerates
the rho = 1 (ordered-subsets SQS) iteration, and the continuation is faster
still.  Measured margins on this workload after 30 iterations (x* from 6000
one-subset iterations): continuation 5.6 HU, rho = 0.05 7.2 HU, rho = 1
11.2 HU; the test uses a shorter x* run, so it checks the order with those
margins, not the values."""
import pytest

from _helpers import ensure_built, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.timeout(300)
def test_rho_sweep_order():
    ensure_built()
    from paper_1402_4381_amd import rho_sweep
    res = rho_sweep.run("fan2d_512", rhos=(1.0, 0.05), iters=30, iters_rho1=30, xstar_iters=2000)
    at30 = res["rmsd_hu_at_30"]
    say("  RMSD at 30 iterations:", at30)
    assert at30["continuation"] < 0.8 * at30["rho=1"]
    assert at30["rho=0.05"] < 0.8 * at30["rho=1"]
    assert at30["continuation"] < at30["rho=0.05"]
