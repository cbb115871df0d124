"""Every launch shape the autotuner can pick (SPME spreading block, y-z plane kernel
slots or one-axis passes) gives the oracle's forces and energies, set by qhp_set_launch."""
import sys

import numpy as np
import pytest

from helpers import has_gpu, medium_box, rel_max
from oracle import forces

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not has_gpu(), reason="needs a HIP device")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


BOXES = {
    # 343 waters, 32^3 grid (four 8^3 tiles along z), P = 16: 8 complex slots
    "k32_p16": dict(P=16, K=32),
    # 64^3 grid, P = 4: 2 complex slots
    "k64_p4": dict(P=4, K=64),
}


@pytest.fixture(scope="module", params=sorted(BOXES))
def case(request):
    s = medium_box(**BOXES[request.param])
    E, F = forces.evaluate(s.pos, s)
    return request.param, s, E, F


def _check(c, s, E_r, F_r, label):
    E, F = c.eval(s.pos)
    err = rel_max(F, F_r)
    assert err <= 1e-11, (label, err)
    assert np.allclose(E, E_r, rtol=1e-11, atol=1e-9), label


def test_spreading_block_shapes(case):
    import paper_2212_03137_amd as q
    name, s, E_r, F_r = case
    nt2 = s.pme_grid[2] // 8
    with q.Context.from_system(s) as c:
        for gb in (1, 2, 4, 8, 16):
            for z in (1, 2, 4, 8):
                if gb * z > 16 or z > nt2 or gb > s.n_beads:
                    continue
                say(name, "spread", gb, z)
                c.set_launch(gb, z, 0)
                _check(c, s, E_r, F_r, (name, gb, z))


def test_plane_kernel_slots_and_one_axis_passes(case):
    import paper_2212_03137_amd as q
    name, s, E_r, F_r = case
    with q.Context.from_system(s) as c:
        for nb in (-1, 1, 2, 4, 8):
            say(name, "fft slots", nb)
            c.set_launch(0, 0, nb)
            _check(c, s, E_r, F_r, (name, nb))


def test_plain_path_on_a_64_point_grid():
    # one bead per launch: the 64^2 plane kernel with one slot
    import paper_2212_03137_amd as q
    s = medium_box(P=2, K=64)
    E_r, F_r = forces.evaluate(s.pos, s)
    with q.Context.from_system(s, exec_mode=q.PLAIN) as c:
        _check(c, s, E_r, F_r, "plain")


def test_set_launch_rejects_bad_shapes():
    import paper_2212_03137_amd as q
    s = medium_box(P=4, K=32)
    with q.Context.from_system(s) as c:
        for bad in ((3, 0, 0), (0, 16, 0), (0, 0, 3), (32, 0, 0), (0, 0, -2)):
            with pytest.raises(q.QhpError) as e:
                c.set_launch(*bad)
            assert e.value.code == q.EINVAL
