"""Every launch shape the autotuner can pick (SPME spreading block, y-z plane kernel
slots or one-axis passes, FP32 pair kernel atoms per block) gives the oracle's forces and
energies, set by qhp_set_launch."""
import sys

import numpy as np
import pytest

from helpers import has_gpu, medium_box, rel_max, rel_rms
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


def test_pair_kernel_atoms_per_block(case):
    # the FP32 pair kernel of the propagation step (no energies) with 2, 4 or 8 atoms per
    # block: each atom's sums do not depend on the block, so three steps from the same
    # state agree up to the order of additions that is not fixed in any case (the order of
    # a cell's atoms, hence of a list row, and the SPME spreading's LDS sums): FP32 force
    # differences of ~1e-7 relative move positions by ~1e-8 A and velocities by ~1e-5 A/ps
    import paper_2212_03137_amd as q
    name, s, E_r, F_r = case
    with q.Context.from_system(s, precision=q.FP32_PAIRS) as c:
        out = {}
        for w in (2, 4, 8):
            say(name, "pair atoms per block", w)
            c.set_launch(0, 0, 0, w)
            c.set_state(s.pos, s.vel, 0)
            c.step(3)
            out[w] = c.get_state()
        x4, v4, _ = out[4]
        for w in (2, 8):
            x, v, st = out[w]
            assert st == 3
            assert rel_max(x, x4) <= 1e-8, (name, w)
            assert rel_max(v, v4) <= 1e-5, (name, w)
        c.set_launch(0, 0, 0, 8)
        E, F = c.eval(s.pos)
    assert rel_rms(F, F_r) <= 1e-5


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
        for bad in ((3, 0, 0, 0), (0, 16, 0, 0), (0, 0, 3, 0), (32, 0, 0, 0), (0, 0, -2, 0),
                    (0, 0, 0, 3), (0, 0, 0, 16), (0, 0, 0, -1)):
            with pytest.raises(q.QhpError) as e:
                c.set_launch(*bad)
            assert e.value.code == q.EINVAL
