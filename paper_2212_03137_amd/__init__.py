"""Python binding of libqhp (the MI355X ring-polymer MD / adaptive QTB library).

Argument marshalling only: every computation runs in the HIP kernels behind the C ABI
declared in ``include/qhp.h``. Importing this package fails loudly when the compiled
library is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqhp.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
MEM_HOST, MEM_DEVICE = 0, 1
FP64, FP32_PAIRS = 0, 1
BATCHED, PLAIN = 0, 1
TRPMD, ADQTB = 0, 1
BAOAB, BCOCB = 0, 1
QTB_SIMPLE, QTB_RATIO = 0, 1
NTERMS = 7
TERMS = ("bond", "angle", "coul_real", "lj", "coul_excl", "coul_self", "coul_recip")
PROF = {"off": 0, "pair": 1, "spread": 2, "fft": 3, "gather": 4, "nm": 5}

EXPORTS = ("qhp_create", "qhp_destroy", "qhp_eval", "qhp_set_state", "qhp_get_state",
           "qhp_step", "qhp_mode_energies", "qhp_nlist_export", "qhp_nlist_stats", "qhp_noise_export",
           "qhp_qtb_get_gamma", "qhp_qtb_set_gamma", "qhp_qtb_get_noise", "qhp_qtb_get_delta",
           "qhp_profile", "qhp_profile_read", "qhp_sync", "qhp_last_error", "qhp_param_grad",
           "qhp_hvp", "qhp_set_lambda", "qhp_eval_lambda", "qhp_bar", "qhp_group_create",
           "qhp_group_step", "qhp_group_destroy", "qhp_group_last_error", "qhp_autotune",
           "qhp_set_launch", "qhp_mode_energies_noalloc")


class QhpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"qhp error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int32), ("n_beads", C.c_int32), ("box", C.c_double * 3),
        ("n_types", C.c_int32), ("type", C.POINTER(C.c_int32)), ("mass", C.POINTER(C.c_double)),
        ("charge", C.POINTER(C.c_double)), ("lj_sigma", C.POINTER(C.c_double)),
        ("lj_epsilon", C.POINTER(C.c_double)),
        ("bond_r0", C.c_double), ("bond_k", C.c_double),
        ("angle_theta0", C.c_double), ("angle_k", C.c_double),
        ("coulomb", C.c_double), ("ewald_alpha", C.c_double), ("cutoff", C.c_double),
        ("skin", C.c_double), ("pme_grid", C.c_int32 * 3), ("pme_order", C.c_int32),
        ("precision", C.c_int32), ("exec", C.c_int32), ("thermostat", C.c_int32),
        ("dt", C.c_double), ("kT", C.c_double), ("hbar", C.c_double),
        ("gamma_centroid", C.c_double), ("trpmd_c", C.c_double), ("seed", C.c_uint64),
        ("qtb_gamma0", C.c_double), ("qtb_nseg", C.c_int32), ("qtb_adapt_rate", C.c_double),
        ("qtb_gamma_min_frac", C.c_double), ("qtb_classical", C.c_int32),
        ("nbr_capacity", C.c_int32), ("use_graph", C.c_int32),
        ("rpc_beads", C.c_int32), ("respa_nalt", C.c_int32),
        ("integrator", C.c_int32), ("qtb_adapt_scheme", C.c_int32), ("qtb_tau", C.c_double),
        ("type_soft", C.POINTER(C.c_int32)), ("lambda_elec", C.c_double),
        ("lambda_vdw", C.c_double), ("sc_alpha", C.c_double),
        ("tether_k", C.c_double), ("tether_anchor", C.POINTER(C.c_double)),
        ("qtb_scheme_of", C.POINTER(C.c_int32)), ("qtb_tau_of", C.POINTER(C.c_double)),
    ]


_lib = None


def load():
    """Load libqhp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with "
                          "`python -m paper_2212_03137_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P, I, D, vp = C.c_void_p, C.c_int, C.POINTER(C.c_double), C.c_void_p
    lib.qhp_create.argtypes = [C.POINTER(Params), vp, C.POINTER(vp)]
    lib.qhp_destroy.argtypes = [vp]
    lib.qhp_eval.argtypes = [vp, vp, vp, vp, vp, I]
    lib.qhp_set_state.argtypes = [vp, vp, vp, C.c_int64, I]
    lib.qhp_get_state.argtypes = [vp, vp, vp, C.POINTER(C.c_int64), I]
    lib.qhp_step.argtypes = [vp, C.c_int32, vp, I]
    lib.qhp_mode_energies.argtypes = [vp, D, D]
    lib.qhp_mode_energies_noalloc.argtypes = [vp, vp]
    lib.qhp_nlist_export.argtypes = [vp, vp, C.c_int64, C.POINTER(C.c_int64)]
    lib.qhp_nlist_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)]
    lib.qhp_noise_export.argtypes = [vp, C.c_int32, C.c_int64, vp]
    lib.qhp_param_grad.argtypes = [vp, vp, vp, vp, vp, I]
    lib.qhp_hvp.argtypes = [vp, vp, vp, vp, vp, vp, vp, I]
    for f in ("qhp_qtb_get_gamma", "qhp_qtb_set_gamma", "qhp_qtb_get_noise", "qhp_qtb_get_delta"):
        getattr(lib, f).argtypes = [vp, vp]
    lib.qhp_profile.argtypes = [vp, I]
    lib.qhp_profile_read.argtypes = [vp, D, C.POINTER(C.c_int64)]
    lib.qhp_set_lambda.argtypes = [vp, C.c_double, C.c_double]
    lib.qhp_eval_lambda.argtypes = [vp, vp, C.c_double, C.c_double, vp, vp, I]
    lib.qhp_bar.argtypes = [vp, C.c_int64, vp, C.c_int64, C.c_double, D, C.POINTER(C.c_int32)]
    lib.qhp_autotune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.qhp_set_launch.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
    lib.qhp_group_create.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(vp)]
    lib.qhp_group_step.argtypes = [vp, C.c_int32]
    lib.qhp_group_destroy.argtypes = [vp]
    lib.qhp_sync.argtypes = [vp]
    lib.qhp_last_error.argtypes = [vp]
    lib.qhp_last_error.restype = C.c_char_p
    lib.qhp_group_last_error.argtypes = [vp]
    lib.qhp_group_last_error.restype = C.c_char_p
    for f in EXPORTS:
        if f not in ("qhp_last_error", "qhp_group_last_error"):
            getattr(lib, f).restype = I
    _lib = lib
    return lib


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    return C.c_void_p(a.data_ptr())      # torch tensor on the device


class Context:
    """One simulation context (owns the device state of P beads of N atoms)."""

    def __init__(self, *, n_atoms, n_beads, box, types, mass, charge, lj_sigma, lj_epsilon,
                 bond_r0, bond_k, angle_theta0, angle_k, coulomb, ewald_alpha, cutoff, skin,
                 pme_grid, pme_order, dt, kT, hbar, gamma_centroid=0.0, trpmd_c=2.0, seed=0,
                 precision=FP64, exec_mode=BATCHED, thermostat=TRPMD, qtb_gamma0=0.0,
                 qtb_nseg=1024, qtb_adapt_rate=0.0, qtb_gamma_min_frac=0.01, qtb_classical=False,
                 nbr_capacity=0, use_graph=True, rpc_beads=0, respa_nalt=1, integrator=0,
                 qtb_adapt_scheme=0, qtb_tau=0.0, type_soft=None, lambda_elec=1.0,
                 lambda_vdw=1.0, sc_alpha=0.5, tether_k=0.0, tether_anchor=None,
                 qtb_scheme_of=None, qtb_tau_of=None, stream=None):
        self._lib = load()
        self.N, self.P = int(n_atoms), int(n_beads)
        self.n_types = len(lj_sigma)
        self.nseg = int(qtb_nseg)
        self._keep = [np.ascontiguousarray(types, dtype=np.int32),
                      np.ascontiguousarray(mass, dtype=np.float64),
                      np.ascontiguousarray(charge, dtype=np.float64),
                      np.ascontiguousarray(lj_sigma, dtype=np.float64),
                      np.ascontiguousarray(lj_epsilon, dtype=np.float64)]
        t, m, q, s, e = self._keep
        p = Params()
        p.n_atoms, p.n_beads = self.N, self.P
        p.box = (C.c_double * 3)(*[float(v) for v in box])
        p.n_types = self.n_types
        p.type = t.ctypes.data_as(C.POINTER(C.c_int32))
        p.mass = m.ctypes.data_as(C.POINTER(C.c_double))
        p.charge = q.ctypes.data_as(C.POINTER(C.c_double))
        p.lj_sigma = s.ctypes.data_as(C.POINTER(C.c_double))
        p.lj_epsilon = e.ctypes.data_as(C.POINTER(C.c_double))
        p.bond_r0, p.bond_k, p.angle_theta0, p.angle_k = bond_r0, bond_k, angle_theta0, angle_k
        p.coulomb, p.ewald_alpha, p.cutoff, p.skin = coulomb, ewald_alpha, cutoff, skin
        p.pme_grid = (C.c_int32 * 3)(*[int(k) for k in pme_grid])
        p.pme_order = pme_order
        p.precision, p.exec, p.thermostat = precision, exec_mode, thermostat
        p.dt, p.kT, p.hbar = dt, kT, hbar
        p.gamma_centroid, p.trpmd_c, p.seed = gamma_centroid, trpmd_c, int(seed)
        p.qtb_gamma0, p.qtb_nseg, p.qtb_adapt_rate = qtb_gamma0, self.nseg, qtb_adapt_rate
        p.qtb_gamma_min_frac, p.qtb_classical = qtb_gamma_min_frac, int(bool(qtb_classical))
        p.nbr_capacity = nbr_capacity
        p.use_graph = int(bool(use_graph))
        p.rpc_beads, p.respa_nalt = int(rpc_beads), int(respa_nalt)
        p.integrator, p.qtb_adapt_scheme, p.qtb_tau = int(integrator), int(qtb_adapt_scheme), qtb_tau
        if type_soft is not None:
            self._keep.append(np.ascontiguousarray(type_soft, dtype=np.int32))
            p.type_soft = self._keep[-1].ctypes.data_as(C.POINTER(C.c_int32))
            p.lambda_elec, p.lambda_vdw, p.sc_alpha = lambda_elec, lambda_vdw, sc_alpha
        p.tether_k = float(tether_k)
        if tether_anchor is not None:
            self._keep.append(np.ascontiguousarray(tether_anchor, dtype=np.float64))
            p.tether_anchor = self._keep[-1].ctypes.data_as(C.POINTER(C.c_double))
        for arr in (qtb_scheme_of, qtb_tau_of):
            if arr is not None and len(arr) != self.n_types:
                raise ValueError("qtb_scheme_of and qtb_tau_of take one entry per type")
        if qtb_scheme_of is not None:
            self._keep.append(np.ascontiguousarray(qtb_scheme_of, dtype=np.int32))
            p.qtb_scheme_of = self._keep[-1].ctypes.data_as(C.POINTER(C.c_int32))
        if qtb_tau_of is not None:
            self._keep.append(np.ascontiguousarray(qtb_tau_of, dtype=np.float64))
            p.qtb_tau_of = self._keep[-1].ctypes.data_as(C.POINTER(C.c_double))
        self.params = p
        h = C.c_void_p()
        rc = self._lib.qhp_create(C.byref(p), C.c_void_p(stream) if stream else None, C.byref(h))
        if rc != OK:
            raise QhpError(rc, "qhp_create failed")
        self._h = h

    @classmethod
    def from_system(cls, s, **kw):
        """Build from any object carrying the fields of ``synth.System``."""
        args = dict(n_atoms=s.n_atoms, n_beads=s.n_beads, box=s.box, types=s.types, mass=s.mass,
                    charge=s.charge, lj_sigma=s.lj_sigma, lj_epsilon=s.lj_epsilon,
                    bond_r0=s.bond_r0, bond_k=s.bond_k, angle_theta0=s.angle_theta0,
                    angle_k=s.angle_k, coulomb=s.coulomb, ewald_alpha=s.ewald_alpha,
                    cutoff=s.cutoff, skin=s.skin, pme_grid=s.pme_grid, pme_order=s.pme_order,
                    dt=s.dt, kT=s.kT, hbar=s.hbar, gamma_centroid=s.gamma_centroid,
                    trpmd_c=s.trpmd_c, seed=s.seed, qtb_gamma0=s.qtb_gamma0,
                    qtb_nseg=s.qtb_nseg, qtb_adapt_rate=s.qtb_adapt_rate,
                    qtb_gamma_min_frac=s.qtb_gamma_min_frac)
        if getattr(s, "type_soft", None) is not None:
            args.update(type_soft=s.type_soft, lambda_elec=s.lambda_elec,
                        lambda_vdw=s.lambda_vdw, sc_alpha=s.sc_alpha)
        if getattr(s, "tether_k", 0.0):
            args.update(tether_k=s.tether_k, tether_anchor=s.tether_anchor)
        args.update(kw)
        return cls(**args)

    # ------------------------------------------------------------------------------
    def _check(self, rc):
        if rc != OK:
            raise QhpError(rc, self._lib.qhp_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.qhp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------------------
    def eval(self, pos, box=None):
        """Per-bead energies [P][7] and forces -grad V [P][N][3] (host arrays); `box` (the
        context's edges, which are fixed per context) is checked when given."""
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        E = np.zeros((self.P, NTERMS))
        F = np.zeros((self.P, self.N, 3))
        b = None if box is None else np.ascontiguousarray(box, dtype=np.float64)
        self._check(self._lib.qhp_eval(self._h, _ptr(pos), _ptr(b), _ptr(E), _ptr(F), MEM_HOST))
        return E, F

    def set_lambda(self, lambda_elec, lambda_vdw):
        """Couplings of the propagated alchemical system (qhp_set_lambda)."""
        self._check(self._lib.qhp_set_lambda(self._h, float(lambda_elec), float(lambda_vdw)))

    def eval_lambda(self, pos, lambda_elec, lambda_vdw, forces=True):
        """qhp_eval of the system at other couplings: energies [P][7] (and forces)."""
        E = np.zeros((self.P, NTERMS))
        F = np.zeros((self.P, self.N, 3)) if forces else None
        if hasattr(pos, "data_ptr"):           # torch tensor on the context's device
            import torch
            Et = torch.zeros((self.P, NTERMS), dtype=torch.float64, device=pos.device)
            self._check(self._lib.qhp_eval_lambda(self._h, _ptr(pos), float(lambda_elec),
                                                  float(lambda_vdw), _ptr(Et), None,
                                                  MEM_DEVICE))
            self.sync()
            return Et.cpu().numpy(), None
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        self._check(self._lib.qhp_eval_lambda(self._h, _ptr(pos), float(lambda_elec),
                                              float(lambda_vdw), _ptr(E), _ptr(F), MEM_HOST))
        return E, F

    def autotune(self, reps=5):
        """Pick the fastest launch shapes for this context (qhp_autotune) -> (beads per
        spreading block, 8^3 tiles along z per spreading block, complex slots per y-z plane
        block or -1 for one-axis passes, FP32 pair kernel atoms per block or 0)."""
        gb, z, nb, w = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self._lib.qhp_autotune(self._h, int(reps), C.byref(gb), C.byref(z),
                                           C.byref(nb), C.byref(w)))
        return gb.value, z.value, nb.value, w.value

    def set_launch(self, spread_beads=0, spread_ztiles=0, fft_slots=0, pair_atoms=0):
        """Launch shapes by hand (qhp_set_launch); 0 = default."""
        self._check(self._lib.qhp_set_launch(self._h, int(spread_beads), int(spread_ztiles),
                                             int(fft_slots), int(pair_atoms)))

    def param_grad(self, pos):
        """d(sum of bead energies) / d(charges [N], lj_epsilon [T], lj_sigma [T])."""
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        dq = np.zeros(self.N)
        de = np.zeros(self.n_types)
        ds = np.zeros(self.n_types)
        self._check(self._lib.qhp_param_grad(self._h, _ptr(pos), _ptr(dq), _ptr(de), _ptr(ds),
                                             MEM_HOST))
        return dq, de, ds

    def hvp(self, pos, direction, mixed=False):
        """Hessian-vector product of every bead's potential, [P][N][3]; with mixed, also
        d(direction . grad E)/d(charges, lj_epsilon, lj_sigma)."""
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        d = np.ascontiguousarray(direction, dtype=np.float64)
        out = np.zeros((self.P, self.N, 3))
        m = [np.zeros(self.N), np.zeros(self.n_types), np.zeros(self.n_types)] if mixed else [None] * 3
        self._check(self._lib.qhp_hvp(self._h, _ptr(pos), _ptr(d), _ptr(out), _ptr(m[0]),
                                      _ptr(m[1]), _ptr(m[2]), MEM_HOST))
        return (out, *m) if mixed else out

    def set_state(self, pos, vel, step=0):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        self._check(self._lib.qhp_set_state(self._h, _ptr(pos), _ptr(vel), int(step), MEM_HOST))

    def get_state(self):
        pos = np.zeros((self.P, self.N, 3))
        vel = np.zeros((self.P, self.N, 3))
        st = C.c_int64()
        self._check(self._lib.qhp_get_state(self._h, _ptr(pos), _ptr(vel), C.byref(st), MEM_HOST))
        return pos, vel, st.value

    def step(self, n=1, energy=False):
        E = np.zeros((self.P, NTERMS)) if energy else None
        self._check(self._lib.qhp_step(self._h, int(n), _ptr(E), MEM_HOST))
        return E

    def mode_energies(self):
        k, s = C.c_double(), C.c_double()
        self._check(self._lib.qhp_mode_energies(self._h, C.byref(k), C.byref(s)))
        return k.value, s.value

    def nlist(self):
        n = C.c_int64()
        self._check(self._lib.qhp_nlist_export(self._h, None, 0, C.byref(n)))
        out = np.zeros((n.value, 2), dtype=np.int32)
        self._check(self._lib.qhp_nlist_export(self._h, _ptr(out), n.value, C.byref(n)))
        return out.astype(np.int64)

    def nlist_stats(self):
        b, m, cap = C.c_int64(), C.c_int32(), C.c_int32()
        self._check(self._lib.qhp_nlist_stats(self._h, C.byref(b), C.byref(m), C.byref(cap)))
        return {"builds": b.value, "max_count": m.value, "capacity": cap.value}

    def noise(self, stream, step):
        rows = self.P if stream == 5 else 1
        out = np.zeros((rows, self.N, 3))
        self._check(self._lib.qhp_noise_export(self._h, int(stream), int(step), _ptr(out)))
        return out if stream == 5 else out[0]

    def qtb_gamma(self):
        out = np.zeros((self.n_types, self.nseg + 1))
        self._check(self._lib.qhp_qtb_get_gamma(self._h, _ptr(out)))
        return out

    def qtb_set_gamma(self, g):
        g = np.ascontiguousarray(g, dtype=np.float64)
        self._check(self._lib.qhp_qtb_set_gamma(self._h, _ptr(g)))

    def qtb_noise(self):
        out = np.zeros((self.nseg, self.N, 3))
        self._check(self._lib.qhp_qtb_get_noise(self._h, _ptr(out)))
        return out

    def qtb_delta(self):
        out = np.zeros((self.n_types, self.nseg + 1))
        self._check(self._lib.qhp_qtb_get_delta(self._h, _ptr(out)))
        return out

    def profile(self, which):
        self._check(self._lib.qhp_profile(self._h, PROF[which] if isinstance(which, str) else which))

    def profile_read(self):
        ms, n = C.c_double(), C.c_int64()
        self._check(self._lib.qhp_profile_read(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def sync(self):
        self._check(self._lib.qhp_sync(self._h))

    # device-memory variants (torch tensors on the context's device)
    def step_device(self, n, energy_tensor=None):
        self._check(self._lib.qhp_step(self._h, int(n), _ptr(energy_tensor), MEM_DEVICE))

    def eval_device(self, pos, energy, forces):
        self._check(self._lib.qhp_eval(self._h, _ptr(pos), None, _ptr(energy), _ptr(forces),
                                       MEM_DEVICE))


def bar(du_a, du_b, beta):
    """Bennett acceptance ratio Delta F_AB (qhp_bar) -> (dF, iterations); du_a, du_b are
    U_B - U_A sampled in states A and B."""
    lib = load()
    a = np.ascontiguousarray(du_a, dtype=np.float64)
    b = np.ascontiguousarray(du_b, dtype=np.float64)
    dF = C.c_double()
    it = C.c_int32()
    rc = lib.qhp_bar(_ptr(a), len(a), _ptr(b), len(b), float(beta), C.byref(dF), C.byref(it))
    if rc != OK:
        raise QhpError(rc, "qhp_bar failed")
    return dF.value, it.value


class Group:
    """Contexts stepped together, one captured graph per step of all members."""

    def __init__(self, contexts):
        self._lib = load()
        self.members = list(contexts)
        arr = (C.c_void_p * len(self.members))(*[c._h.value for c in self.members])
        h = C.c_void_p()
        rc = self._lib.qhp_group_create(arr, len(self.members), C.byref(h))
        if rc != OK:
            raise QhpError(rc, "qhp_group_create failed")
        self._h = h

    def step(self, nsteps=1):
        rc = self._lib.qhp_group_step(self._h, int(nsteps))
        if rc != OK:
            raise QhpError(rc, self._lib.qhp_group_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.qhp_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
