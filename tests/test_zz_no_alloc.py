"""The allocation-free entry point qhp_mode_energies_noalloc against qhp_mode_energies,
called through the C ABI: two calls in a row on the same GPU, the second on a smaller
system (fewer blocks of partial sums than the first left in the shared scratch).

Bar: both are FP64 sums of the same per-lane terms in a different order, so they agree to
1e-12 relative."""
import ctypes as C
import math

import numpy as np
import pytest

import synth
from helpers import has_gpu

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not has_gpu(), reason="needs a HIP device")]


def _both(s, steps, **kw):
    import torch
    import paper_2212_03137_amd as q
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    with q.Context.from_system(s, **kw) as c:
        c.set_state(s.pos, s.vel, 0)
        c.step(steps)
        kin, spr = c.mode_energies()
        rc = c._lib.qhp_mode_energies_noalloc(c._h, C.c_void_p(out.data_ptr()))
        assert rc == q.OK, c._lib.qhp_last_error(c._h)
        c.sync()
        got = out.cpu().numpy()
    return (kin, spr), got


@pytest.mark.parametrize("respa", [False, True])
def test_noalloc_mode_energies_match_the_allocating_call(respa):
    big = synth.large_rpmd()                               # 1,536 blocks of partial sums
    small = synth.small_rpmd()                             # 6 blocks
    kw = dict(rpc_beads=4, respa_nalt=2) if respa else {}
    for s, steps in ((big, 3), (small, 5)):
        (kin, spr), got = _both(s, steps, **kw)
        print("noalloc", s.name, kin, spr, got, flush=True)
        assert math.isclose(got[0], kin, rel_tol=1e-12)
        assert math.isclose(got[1], spr, rel_tol=1e-12)


def test_noalloc_needs_a_state_and_an_output():
    import paper_2212_03137_amd as q
    s = synth.small_rpmd()
    with q.Context.from_system(s) as c:
        assert c._lib.qhp_mode_energies_noalloc(c._h, None) == q.EINVAL
        assert c._lib.qhp_mode_energies_noalloc(c._h, C.c_void_p(8)) == q.EINVAL   # no state
