"""The C-ABI library loads and exports every entry point the header declares; argument
validation happens before any device call, so it is testable without a GPU."""
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "qhp.h")).read()
    return sorted(set(re.findall(r"QHP_API\s+(?:int|const char\*)\s+(qhp_\w+)\s*\(", src)))


def test_header_declares_the_binding_surface():
    import paper_2212_03137_amd as q
    assert sorted(q.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    import ctypes
    import paper_2212_03137_amd as q
    if not os.path.exists(q.LIB_PATH):
        pytest.skip("libqhp.so not built")
    lib = ctypes.CDLL(q.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_params_struct_matches_header_fields():
    import paper_2212_03137_amd as q
    src = open(os.path.join(ROOT, "include", "qhp.h")).read()
    body = src[src.index("typedef struct qhp_params {"):src.index("} qhp_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)          # comments
    fields = re.findall(r"^\s*(?:const\s+)?[\w]+\**\s+\**([\w, ]+?)(?:\[\d\])?;", body, flags=re.M)
    names = []
    for f in fields:
        names += [n.strip() for n in f.split(",")]
    assert names == [f[0] for f in q.Params._fields_]


@pytest.mark.parametrize("change,code", [
    (dict(cutoff=7.0), -1),            # rc >= L/2 for a 12.42 A box
    (dict(n_beads=65), -1),            # more than 64 beads
    (dict(pme_order=7), -5),
    (dict(pme_grid=(16, 16, 12)), -1),
    (dict(exec_mode=7), -1),
    (dict(tether_k=-1.0), -1),         # the test tether: k_h >= 0
    (dict(tether_k=2.0), -1),          # k_h > 0 without anchors
])
def test_invalid_parameters_rejected_before_device_use(change, code):
    import paper_2212_03137_amd as q
    if not os.path.exists(q.LIB_PATH):
        pytest.skip("libqhp.so not built")
    s = synth.small_rpmd()
    with pytest.raises(q.QhpError) as e:
        q.Context.from_system(s, **change)
    assert e.value.code == code


@pytest.mark.parametrize("change,code", [
    (dict(qtb_scheme_of=[0, 1], qtb_tau_of=[1.0, 0.0]), -1),   # a RATIO type without a time
    (dict(qtb_scheme_of=[0, 7]), -1),                           # no such scheme
    (dict(qtb_scheme_of=[0, 1], qtb_tau_of=[0.0, 1.0]), None),  # a SIMPLE type needs none
    (dict(qtb_adapt_scheme=1, qtb_tau_of=[5.0, 1.0]), None),    # every type RATIO, own times
])
def test_per_type_adaptation_validated_before_device_use(change, code):
    # the adQTB per-type schemes and times; a valid set reaches the device (which this
    # container lacks: QHP_EDEVICE)
    import paper_2212_03137_amd as q
    if not os.path.exists(q.LIB_PATH):
        pytest.skip("libqhp.so not built")
    s = synth.water_box(27, 1, 12.0, seed=9, cutoff=5.5, ewald_alpha=0.4, pme_grid=16,
                        pme_order=4, qtb_gamma0=0.02, qtb_nseg=32, qtb_adapt_rate=1e-3)
    try:
        c = q.Context.from_system(s, thermostat=q.ADQTB, **change)
    except q.QhpError as e:
        assert e.code == (q.EINVAL if code is not None else q.EDEVICE), e.code
    else:
        c.close()
        assert code is None
    with pytest.raises(ValueError):
        q.Context.from_system(s, thermostat=q.ADQTB, qtb_tau_of=[1.0])


@pytest.mark.parametrize("nseg,ok", [(8, False), (20, False), (88, False), (2048, False),
                                     (24, True), (120, True), (1000, True), (1024, True)])
def test_segment_lengths_validated_before_device_use(nseg, ok):
    # N_seg: 16..1024, a multiple of 8, prime factors 2, 3, 5, 7 only (88 = 8 x 11 is not)
    import paper_2212_03137_amd as q
    if not os.path.exists(q.LIB_PATH):
        pytest.skip("libqhp.so not built")
    s = synth.water_box(27, 1, 12.0, seed=9, cutoff=5.5, ewald_alpha=0.4, pme_grid=16,
                        pme_order=4, qtb_gamma0=0.02, qtb_nseg=nseg, qtb_adapt_rate=1e-3)
    try:
        c = q.Context.from_system(s, thermostat=q.ADQTB)
    except q.QhpError as e:
        assert e.code == (q.EDEVICE if ok else q.EINVAL), e.code
    else:
        c.close()
        assert ok


@pytest.mark.parametrize("grid,code", [((24, 24, 24), "device"), ((40, 16, 56), "device"),
                                       ((20, 16, 16), "inval"), ((88, 16, 16), "inval"),
                                       ((136, 16, 16), "inval")])
def test_spme_grids_validated_before_device_use(grid, code):
    # grid edges: powers of two, or multiples of 8 with prime factors 2, 3, 5, 7, up to 128
    import dataclasses
    import paper_2212_03137_amd as q
    if not os.path.exists(q.LIB_PATH):
        pytest.skip("libqhp.so not built")
    s = dataclasses.replace(synth.small_rpmd(), pme_grid=grid)
    with pytest.raises(q.QhpError) as e:
        q.Context.from_system(s)
    assert e.value.code == (q.EDEVICE if code == "device" else q.EINVAL), e.value.code
    if code == "device":
        with pytest.raises(q.QhpError) as e:
            q.Context.from_system(s, exec_mode=q.PLAIN)
        assert e.value.code == q.EDEVICE
