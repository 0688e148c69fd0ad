"""ctypes binding of libuseries.so: the C ABI declared in include/useries.h.

Argument marshalling only; every step of an evaluation runs in the
library's HIP kernels.  The functions keep the C names.  Device buffers are
passed as integer addresses (e.g. ``tensor.data_ptr()``), streams as the
integer value of a hipStream_t (``torch.cuda.current_stream().cuda_stream``).
If the library has not been built, loading fails loudly: there is no
fallback implementation.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libuseries.so")

USERIES_OK = 0
USERIES_EINVAL = -1
USERIES_ENOMEM = -2
USERIES_EHIP = -3
USERIES_EBUSY = -4
USERIES_ENOTFOUND = -5
USERIES_ESTATE = -6

USERIES_C0 = 0
USERIES_C1 = 1
USERIES_C2_B2 = 2
USERIES_TABLE1_ROW1 = 11
USERIES_TABLE1_ROW2 = 12
USERIES_TABLE1_ROW3 = 13

USERIES_PLAIN_FP32 = 0
USERIES_BF16X3 = 1

# every symbol include/useries.h declares
EXPORTED = [
    "useries_default_opts", "useries_plan", "useries_eval", "useries_eval_parts",
    "useries_plan_info", "useries_destroy", "useries_timing_enable", "useries_timing_read",
    "useries_solve_construction", "useries_eq33_bound", "useries_choose_nterms",
    "useries_bsa_bound", "useries_strerror", "useries_last_error",
]


class UseriesError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_strerror(code), code, msg))
        self.code = code


class useries_opts(ctypes.Structure):
    _fields_ = [("construction", ctypes.c_int), ("precision", ctypes.c_int),
                ("sigma_s_over_h", ctypes.c_double), ("stencil_half", ctypes.c_int),
                ("nterms_tol", ctypes.c_double), ("poly_degree", ctypes.c_int),
                ("max_atoms", ctypes.c_int64)]


_lib = None


def lib():
    """The loaded library; raises if it is missing (build() first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libuseries.so is not built (%s): call __graft_entry__.build() or "
                           "python -m paper_1911_01377_amd._build" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    I, D, P, I64 = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_int64
    sig = {
        "useries_default_opts": (I, [P]),
        "useries_plan": (I, [P, P, D, D, D, I, P, P]),
        "useries_eval": (I, [P, I64, P, P, P, P, P]),
        "useries_eval_parts": (I, [P, I64, P, P, P, P, P, P]),
        "useries_plan_info": (I, [P] + [P] * 13),
        "useries_destroy": (I, [P]),
        "useries_timing_enable": (I, [P, I]),
        "useries_timing_read": (I, [P, I, P, P, P]),
        "useries_solve_construction": (I, [I, D, P, P, P, P]),
        "useries_eq33_bound": (D, [I, D, D, D]),
        "useries_choose_nterms": (I, [D, D, D, D]),
        "useries_bsa_bound": (D, [D]),
        "useries_strerror": (ctypes.c_char_p, [I]),
        "useries_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _strerror(code):
    try:
        return lib().useries_strerror(code).decode()
    except Exception:
        return "error"


def _check(code):
    if code != USERIES_OK:
        raise UseriesError(code, lib().useries_last_error().decode())
    return code


def _d3(v):
    return (ctypes.c_double * 3)(*[float(x) for x in v])


def _i3(v):
    return (ctypes.c_int * 3)(*[int(x) for x in v])


# ----------------------------------------------------------------- C names

def useries_default_opts():
    o = useries_opts()
    _check(lib().useries_default_opts(ctypes.byref(o)))
    return o


def useries_plan(box, r_c, b, sigma, n_terms, grid, opts=None):
    """Returns the plan handle (an opaque pointer value)."""
    h = ctypes.c_void_p()
    _check(lib().useries_plan(ctypes.byref(h), _d3(box), float(r_c), float(b), float(sigma),
                              int(n_terms), _i3(grid),
                              ctypes.byref(opts) if opts is not None else None))
    return h.value


def useries_eval(plan, n, xyz, q, forces, energy, stream=0):
    _check(lib().useries_eval(plan, int(n), xyz, q, forces, energy, stream or None))


def useries_eval_parts(plan, n, xyz, q, forces, energy, parts, stream=0):
    _check(lib().useries_eval_parts(plan, int(n), xyz, q, forces, energy or None, parts,
                                    stream or None))


def useries_plan_info(plan):
    vals = [ctypes.c_double() for _ in range(5)]
    nt = ctypes.c_int()
    eq33, f0, slope, ss, perr = (ctypes.c_double() for _ in range(5))
    P = ctypes.c_int()
    nc = (ctypes.c_int * 3)()
    _check(lib().useries_plan_info(plan, *[ctypes.byref(v) for v in vals], ctypes.byref(nt),
                                   ctypes.byref(eq33), ctypes.byref(f0), ctypes.byref(slope),
                                   ctypes.byref(ss), ctypes.byref(P), nc, ctypes.byref(perr)))
    b, sigma, r0, w0, s0 = (v.value for v in vals)
    return dict(b=b, sigma=sigma, r0=r0, w0=w0, s0=s0, n_terms=nt.value, eq33=eq33.value,
                f_inf0=f0.value, c1_slope=slope.value, sigma_s=ss.value,
                stencil_half=P.value, ncell=tuple(nc), poly_maxerr=perr.value)


def useries_destroy(plan):
    _check(lib().useries_destroy(plan))


def useries_timing_enable(plan, enable):
    _check(lib().useries_timing_enable(plan, int(bool(enable))))


def useries_timing_read(plan):
    """[(kernel name, total ms, launches)] in launch order."""
    out = []
    k = 0
    while True:
        name = ctypes.c_char_p()
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        rc = lib().useries_timing_read(plan, k, ctypes.byref(name), ctypes.byref(ms),
                                       ctypes.byref(cnt))
        if rc == USERIES_ENOTFOUND:
            return out
        _check(rc)
        out.append((name.value.decode(), ms.value, cnt.value))
        k += 1


def useries_solve_construction(construction, b=2.0):
    bo, r0, w0, s0 = (ctypes.c_double() for _ in range(4))
    _check(lib().useries_solve_construction(int(construction), float(b), ctypes.byref(bo),
                                            ctypes.byref(r0), ctypes.byref(w0), ctypes.byref(s0)))
    return bo.value, r0.value, w0.value, s0.value


def useries_eq33_bound(n, b, sigma, lmax):
    return lib().useries_eq33_bound(int(n), float(b), float(sigma), float(lmax))


def useries_choose_nterms(b, sigma, lmax, tol):
    return lib().useries_choose_nterms(float(b), float(sigma), float(lmax), float(tol))


def useries_bsa_bound(b):
    return lib().useries_bsa_bound(float(b))


def useries_strerror(code):
    return _strerror(code)


def useries_last_error():
    return lib().useries_last_error().decode()


__all__ = [n for n in dir() if n.startswith(("useries_", "USERIES_"))] + ["lib", "UseriesError"]
