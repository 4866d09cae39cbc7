"""lbm_diagnostics_noalloc (reduction scratch in the library's static device
array) against lbm_diagnostics (scratch in the workspace), through the C ABI:
the same kernels in the same order, so the sums must be bit-identical.  Two
calls in a row on two contexts, the second on a smaller domain, so the
second call reads a scratch the first left behind; then a third call back on
the first context."""
import numpy as np
import pytest

from paper_2506_21804_amd import inputs as I
from gpu_helpers import announce

pytestmark = pytest.mark.gpu


def test_diagnostics_noalloc_matches_workspace_reduction(gpu):
    big = gpu.Lattice(I.channel(96, 48, 40, q=27), storage="f32")
    small = gpu.Lattice(I.taylor_green(12, q=19), storage="f64")
    big.step(3)
    small.step(2)
    for name, lat in (("channel 96x48x40 f32", big), ("tgv 12^3 f64", small), ("channel again", big)):
        announce(f"noalloc diagnostics: {name}")
        a = gpu.lbm_diagnostics_noalloc(lat.ctx)
        b = gpu.lbm_diagnostics(lat.ctx)
        announce(f"{name}: noalloc {a.tolist()} workspace {b.tolist()}")
        assert np.array_equal(a, b), (a, b)
    assert small.diagnostics()[0] == pytest.approx(12 ** 3, rel=1e-12)
