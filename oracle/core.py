"""ctypes wrapper of the FP64 u-series oracle (``useries_oracle.c``).

TEST INFRASTRUCTURE ONLY: see the package docstring.  Every function takes
and returns float64 numpy arrays; positions are ``[n, 3]`` in Angstrom,
charges ``[n]`` in e, the box is the three edge lengths of the orthorhombic
cell.  The physics and the citations of the paper are in the C source.
"""
import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "useries_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


@dataclass
class Params:
    """u-series parameters: base b, width sigma, narrowest weight w0 (eq. 24),
    narrowest width factor s0 (eq. 28), cutoff r_c, far terms N (Sec. V), and
    the power alpha of the kernel 1/r^alpha (App. A; 1 = Coulomb)."""
    b: float
    sigma: float
    w0: float
    s0: float
    rc: float
    nterms: int
    alpha: float = 1.0


class _CParams(ctypes.Structure):
    _fields_ = [("b", ctypes.c_double), ("sigma", ctypes.c_double), ("w0", ctypes.c_double),
                ("s0", ctypes.c_double), ("rc", ctypes.c_double), ("nterms", ctypes.c_int),
                ("alpha", ctypes.c_double)]


def _cp(p):
    return ctypes.byref(_CParams(p.b, p.sigma, p.w0, p.s0, p.rc, int(p.nterms),
                                 float(getattr(p, "alpha", 1.0))))


def build(force=True):
    """Compile liboracle.so with gcc (plain -O2, IEEE arithmetic, OpenMP)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    D, I, P = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
    sig = {
        "uo_series_len": (I, [D]),
        "uo_term": (None, [P, I, P, P]),
        "uo_far_inf": (None, [P, D, P]),
        "uo_near": (None, [P, D, P]),
        "uo_bsa_bound": (D, [D]),
        "uo_eq33_bound": (D, [I, D, D, D]),
        "uo_c1_w0": (D, [D, D]),
        "uo_solve_c0": (I, [D, P]),
        "uo_solve_c1": (I, [D, P, P]),
        "uo_far_inf0": (D, [P]),
        "uo_near_integral": (D, [P]),
        "uo_eval": (I, [I, P, P, P, P, P, P]),
        "uo_eval_near": (I, [I, P, P, P, P, P, P]),
        "uo_eval_far": (I, [I, P, P, P, P, P, P]),
        "uo_forces_subset": (I, [I, P, P, P, P, I, P, P]),
        "uo_far_kspace": (I, [I, P, P, P, P, P, P]),
        "uo_num_threads": (I, []),
        "uo_mellin_gauss": (D, [D]),
        "uo_trunc_bound": (D, [I, D, D, D, D]),
        "uo_c1_w0a": (D, [D, D, D]),
        "uo_solve_c1a": (I, [D, D, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _arr(x, shape=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _inputs(xyz, q, box):
    xyz = _arr(xyz).reshape(-1, 3)
    q = _arr(q).reshape(-1)
    box = _arr(box).reshape(3)
    if xyz.shape[0] != q.shape[0]:
        raise ValueError("xyz and q disagree on the number of charges")
    return xyz, q, box


def series_len(b):
    return load().uo_series_len(b)


def term(p, j):
    """(a_j, s_j) of Gaussian term j."""
    a, s = ctypes.c_double(), ctypes.c_double()
    load().uo_term(_cp(p), j, ctypes.byref(a), ctypes.byref(s))
    return a.value, s.value


def far_inf(p, r):
    """F_inf(r), F_inf'(r), F_inf''(r) (all series terms)."""
    out = np.zeros(3)
    load().uo_far_inf(_cp(p), float(r), _ptr(out))
    return out


def near_kernel(p, r):
    """N(r) of eq. 20 and N'(r)."""
    out = np.zeros(2)
    load().uo_near(_cp(p), float(r), _ptr(out))
    return out


def far_inf0(p):
    return load().uo_far_inf0(_cp(p))


def near_integral(p):
    return load().uo_near_integral(_cp(p))


def bsa_bound(b):
    return load().uo_bsa_bound(b)


def eq33_bound(n, b, sigma, lmax):
    return load().uo_eq33_bound(int(n), b, sigma, lmax)


def c1_w0(b, r):
    return load().uo_c1_w0(b, r)


def solve_c0(b):
    r0 = ctypes.c_double()
    if load().uo_solve_c0(b, ctypes.byref(r0)):
        raise RuntimeError("no C0 root found")
    return r0.value


def solve_c1(b):
    r0, w0 = ctypes.c_double(), ctypes.c_double()
    if load().uo_solve_c1(b, ctypes.byref(r0), ctypes.byref(w0)):
        raise RuntimeError("no C1 root found")
    return r0.value, w0.value


def mellin_gauss(alpha):
    """phi~(alpha) of eq. A1 for the unit Gaussian."""
    return load().uo_mellin_gauss(float(alpha))


def trunc_bound(n, b, alpha, sigma, lmax):
    """Truncation bound of the 1/r^alpha far part at n terms (eq. 33 at alpha = 1)."""
    return load().uo_trunc_bound(int(n), float(b), float(alpha), float(sigma), float(lmax))


def c1_w0a(b, alpha, r):
    """w0 of the C1 construction for 1/r^alpha at r (sigma = 1)."""
    return load().uo_c1_w0a(float(b), float(alpha), float(r))


def solve_c1a(b, alpha):
    """(r0, w0) of the C1 construction for 1/r^alpha."""
    r0, w0 = ctypes.c_double(), ctypes.c_double()
    if load().uo_solve_c1a(float(b), float(alpha), ctypes.byref(r0), ctypes.byref(w0)):
        raise RuntimeError("no C1 root found")
    return r0.value, w0.value


def num_threads():
    return load().uo_num_threads()


def eval_full(xyz, q, box, p):
    """Returns (parts, forces): parts = dict(near, far, self, bg, total)."""
    xyz, q, box = _inputs(xyz, q, box)
    n = q.shape[0]
    f = np.zeros((n, 3))
    parts = np.zeros(5)
    if load().uo_eval(n, _ptr(xyz), _ptr(q), _ptr(box), _cp(p), _ptr(f), _ptr(parts)):
        raise ValueError("invalid parameters")
    return dict(near=parts[0], far=parts[1], self=parts[2], bg=parts[3], total=parts[4]), f


def eval_near(xyz, q, box, p):
    xyz, q, box = _inputs(xyz, q, box)
    n = q.shape[0]
    f = np.zeros((n, 3))
    e = np.zeros(1)
    load().uo_eval_near(n, _ptr(xyz), _ptr(q), _ptr(box), _cp(p), _ptr(f), _ptr(e))
    return e[0], f


def eval_far(xyz, q, box, p):
    xyz, q, box = _inputs(xyz, q, box)
    n = q.shape[0]
    f = np.zeros((n, 3))
    e = np.zeros(1)
    load().uo_eval_far(n, _ptr(xyz), _ptr(q), _ptr(box), _cp(p), _ptr(f), _ptr(e))
    return e[0], f


def far_kspace(xyz, q, box, p):
    xyz, q, box = _inputs(xyz, q, box)
    n = q.shape[0]
    f = np.zeros((n, 3))
    e = np.zeros(1)
    if load().uo_far_kspace(n, _ptr(xyz), _ptr(q), _ptr(box), _cp(p), _ptr(f), _ptr(e)):
        raise ValueError("invalid parameters")
    return e[0], f


def forces_subset(xyz, q, box, p, idx):
    """Total (near + far) forces on atoms idx only, each by its own O(n) sum."""
    xyz, q, box = _inputs(xyz, q, box)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int32))
    out = np.zeros((idx.shape[0], 3))
    if load().uo_forces_subset(q.shape[0], _ptr(xyz), _ptr(q), _ptr(box), _cp(p),
                               idx.shape[0], idx.ctypes.data_as(ctypes.c_void_p), _ptr(out)):
        raise ValueError("invalid parameters")
    return out
