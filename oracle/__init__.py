"""Test infrastructure: the CPU oracle of the cloning algorithm.

Only the tests, the smoke check and the CPU baseline leg of the benchmark may
import this package.  It wraps ``oracle.c`` (a plain C, FP64, sequential
implementation of the algorithm of arXiv:1711.05095, Secs. 2.3, 3 and 4) and
holds the exact-diagonalisation checker in :mod:`oracle.ed`.  It shares no code
with the GPU library.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODIFIED, DIRECT, GUIDED = 0, 1, 2
SEL_EQ, SEL_IID = 0, 1


def build(force=False):
    """Compile oracle.c with gcc (no FP contraction, so fma appears only where
    the source writes it)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-shared",
                               "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("N", ctypes.c_int32), ("s", ctypes.c_double),
                ("Nc", ctypes.c_int64), ("dt", ctypes.c_double), ("M", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("instance", ctypes.c_uint32),
                ("mode", ctypes.c_int32), ("selection", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("burn_in", ctypes.c_int64),
                ("guide", ctypes.POINTER(ctypes.c_uint32))]


class Result(ctypes.Structure):
    _fields_ = [("psi", ctypes.c_double), ("psi_burn", ctypes.c_double),
                ("k_hat", ctypes.c_double), ("hops", ctypes.c_uint64),
                ("cycles", ctypes.c_int64), ("k_hat_burn", ctypes.c_double)]


_lib = None


def lib():
    """The compiled oracle.  PD_ORACLE_LIB, when set, names another build of it
    to load instead (the test that plants mistakes in copies of oracle.c runs
    the pins against each copy this way)."""
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(os.environ.get("PD_ORACLE_LIB") or build())
        P = ctypes.POINTER
        _lib.orc_philox.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        _lib.orc_init.argtypes = [P(Params), ctypes.c_void_p, ctypes.c_void_p]
        _lib.orc_step.argtypes = [P(Params), ctypes.c_uint32] + [ctypes.c_void_p] * 5
        _lib.orc_eq_offset.argtypes = [P(Params), ctypes.c_uint32]
        _lib.orc_eq_offset.restype = ctypes.c_double
        _lib.orc_select.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
        _lib.orc_select.restype = ctypes.c_double
        _lib.orc_resample.argtypes = [P(Params), ctypes.c_uint32] + [ctypes.c_void_p] * 6
        _lib.orc_resample.restype = ctypes.c_double
        _lib.orc_run.argtypes = [P(Params), P(Result), ctypes.c_void_p, ctypes.c_void_p]
        _lib.orc_run_lineage.argtypes = [P(Params), ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]
        _lib.orc_step_slots.argtypes = [P(Params), ctypes.c_uint32, ctypes.c_int64] + \
            [ctypes.c_void_p] * 6
        _lib.orc_iid_points.argtypes = [P(Params), ctypes.c_uint32, ctypes.c_void_p]
        _lib.orc_init_slots.argtypes = [P(Params), ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.c_void_p]
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """One parameter set of the algorithm.  Populations are held as numpy
    arrays: ``occ`` uint8 [Nc, L] (site occupancies) and ``K`` uint64 [Nc]."""

    def __init__(self, L, N, s, Nc, dt, M=1, seed=0, instance=0, mode=MODIFIED,
                 selection=SEL_EQ, burn_in=0, guide=None):
        self.p = Params(L=L, N=N, s=float(s), Nc=Nc, dt=float(dt), M=M, seed=seed,
                        instance=instance, mode=mode, selection=selection, pad_=0,
                        burn_in=burn_in)
        self._guide = None
        if guide is not None:
            self._guide = np.ascontiguousarray(guide, dtype=np.uint32)
            assert self._guide.shape == (8192,)
            self.p.guide = self._guide.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        self.L, self.N, self.Nc = L, N, Nc

    def init(self):
        occ = np.zeros((self.Nc, self.L), np.uint8)
        K = np.zeros(self.Nc, np.uint64)
        lib().orc_init(ctypes.byref(self.p), _ptr(occ), _ptr(K))
        return occ, K

    def step(self, beta, occ, K):
        """Dynamical stage of interval beta, in place on occ and K.
        Returns (Kb, A, ell)."""
        assert occ.dtype == np.uint8 and occ.shape == (self.Nc, self.L) and occ.flags.c_contiguous
        assert K.dtype == np.uint64 and K.shape == (self.Nc,)
        Kb = np.zeros(self.Nc, np.uint32)
        A = np.zeros(self.Nc, np.float64)
        ell = np.zeros(self.Nc, np.float64)
        lib().orc_step(ctypes.byref(self.p), beta, _ptr(occ), _ptr(K), _ptr(Kb), _ptr(A),
                       _ptr(ell))
        return Kb, A, ell

    def step_slots(self, beta, slots, occ, K):
        """Dynamical stage for the clones in the given slots only (occ[i] is the
        clone of slot slots[i]); in place.  Returns (Kb, A, ell)."""
        slots = np.ascontiguousarray(slots, np.int64)
        n = slots.shape[0]
        assert occ.dtype == np.uint8 and occ.shape == (n, self.L) and occ.flags.c_contiguous
        Kb = np.zeros(n, np.uint32)
        A = np.zeros(n, np.float64)
        ell = np.zeros(n, np.float64)
        lib().orc_step_slots(ctypes.byref(self.p), beta, n, _ptr(slots), _ptr(occ), _ptr(K),
                             _ptr(Kb), _ptr(A), _ptr(ell))
        return Kb, A, ell

    def init_slots(self, slots):
        slots = np.ascontiguousarray(slots, np.int64)
        occ = np.zeros((slots.shape[0], self.L), np.uint8)
        lib().orc_init_slots(ctypes.byref(self.p), slots.shape[0], _ptr(slots), _ptr(occ))
        return occ

    def iid_points(self, beta):
        """The [iid] points of interval beta, in units of the point spacing."""
        pts = np.empty(self.Nc, np.float64)
        lib().orc_iid_points(ctypes.byref(self.p), beta, _ptr(pts))
        return pts

    def eq_offset(self, beta):
        return lib().orc_eq_offset(ctypes.byref(self.p), beta)

    def resample(self, beta, occ, K, ell):
        """Cloning stage of interval beta.  Returns (occ_new, K_new, anc, ln mean Ups)."""
        occ2 = np.empty_like(occ)
        K2 = np.empty_like(K)
        anc = np.empty(self.Nc, np.int32)
        ell = np.ascontiguousarray(ell, np.float64)
        lm = lib().orc_resample(ctypes.byref(self.p), beta, _ptr(occ), _ptr(K), _ptr(ell),
                                _ptr(occ2), _ptr(K2), _ptr(anc))
        return occ2, K2, anc, lm

    def run(self, per_interval=False):
        res = Result()
        M = self.p.M
        lb = np.zeros(M) if per_interval else None
        mk = np.zeros(M) if per_interval else None
        rc = lib().orc_run(ctypes.byref(self.p), ctypes.byref(res),
                           _ptr(lb) if per_interval else None,
                           _ptr(mk) if per_interval else None)
        if rc != 0:
            raise MemoryError("oracle run failed")
        out = dict(psi=res.psi, psi_burn=res.psi_burn, k_hat=res.k_hat,
                   k_hat_burn=res.k_hat_burn, hops=res.hops, cycles=res.cycles)
        if per_interval:
            out["lbeta"] = lb
            out["mean_kb"] = mk
        return out

    def run_lineage(self, beta0):
        """Whole run with origins carried from interval beta0 on.  Returns
        (occ at beta0 after cloning, final occ, origin of every final clone)."""
        occ0 = np.zeros((self.Nc, self.L), np.uint8)
        occ1 = np.zeros((self.Nc, self.L), np.uint8)
        org = np.zeros(self.Nc, np.int32)
        rc = lib().orc_run_lineage(ctypes.byref(self.p), int(beta0), _ptr(occ0), _ptr(occ1),
                                   _ptr(org))
        if rc != 0:
            raise ValueError("oracle lineage run failed (%d)" % rc)
        return occ0, occ1, org


def select(ell, d=None, points=None):
    """Selection alone: [eq] with offset d, or [iid] with points (in units of
    the spacing).  Returns (anc, ln mean Upsilon)."""
    ell = np.ascontiguousarray(ell, np.float64)
    Nc = ell.shape[0]
    anc = np.empty(Nc, np.int32)
    if points is None:
        lm = lib().orc_select(Nc, _ptr(ell), SEL_EQ, float(d), None, _ptr(anc))
    else:
        pts = np.ascontiguousarray(points, np.float64)
        lm = lib().orc_select(Nc, _ptr(ell), SEL_IID, 0.0, _ptr(pts), _ptr(anc))
    return anc, lm


def philox(ctr, key):
    """One Philox4x32-10 block."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox(c, k, o)
    return list(o)
