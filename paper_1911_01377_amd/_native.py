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

USERIES_PENDING = 0
USERIES_RUNNING = 1
USERIES_DONE = 2
USERIES_ERROR = 3

# every symbol include/useries.h declares
EXPORTED = [
    "useries_default_opts", "useries_plan", "useries_eval", "useries_eval_parts",
    "useries_plan_info", "useries_destroy", "useries_timing_enable", "useries_timing_read",
    "useries_solve_construction", "useries_eq33_bound", "useries_choose_nterms",
    "useries_bsa_bound", "useries_strerror", "useries_last_error",
    "useries_server_default_opts", "useries_server_create", "useries_submit", "useries_poll",
    "useries_wait", "useries_request_times", "useries_server_stats", "useries_server_destroy",
    "useries_server_hold",
    "useries_philox4x32_10",
    "useries_eval_static",
]


class UseriesError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_strerror(code), code, msg))
        self.code = code


class useries_opts(ctypes.Structure):
    _fields_ = [("construction", ctypes.c_int), ("precision", ctypes.c_int),
                ("sigma_s_over_h", ctypes.c_double), ("stencil_half", ctypes.c_int),
                ("nterms_tol", ctypes.c_double), ("poly_degree", ctypes.c_int),
                ("max_atoms", ctypes.c_int64), ("alpha", ctypes.c_int),
                ("spectral", ctypes.c_int)]


class useries_request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("xyz", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("box", ctypes.c_double * 3), ("r_c", ctypes.c_double),
                ("grid", ctypes.c_int * 3), ("n_evals", ctypes.c_int),
                ("disp_sigma", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("energies", ctypes.c_void_p), ("forces", ctypes.c_void_p),
                ("xyz_final", ctypes.c_void_p)]


class useries_server_opts(ctypes.Structure):
    _fields_ = [("construction", ctypes.c_int), ("b", ctypes.c_double),
                ("nterms_tol", ctypes.c_double), ("poly_degree", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("inflight", ctypes.c_int)]


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
        "useries_plan_info": (I, [P] + [P] * 17),
        "useries_destroy": (I, [P]),
        "useries_timing_enable": (I, [P, I]),
        "useries_timing_read": (I, [P, I, P, P, P]),
        "useries_solve_construction": (I, [I, D, P, P, P, P]),
        "useries_eq33_bound": (D, [I, D, D, D]),
        "useries_choose_nterms": (I, [D, D, D, D]),
        "useries_bsa_bound": (D, [D]),
        "useries_strerror": (ctypes.c_char_p, [I]),
        "useries_last_error": (ctypes.c_char_p, []),
        "useries_server_default_opts": (I, [P]),
        "useries_server_create": (I, [P, ctypes.c_size_t, I, I, P]),
        "useries_submit": (I, [P, P, P]),
        "useries_poll": (I, [P, ctypes.c_uint64, P]),
        "useries_wait": (I, [P, ctypes.c_uint64, P]),
        "useries_request_times": (I, [P, ctypes.c_uint64, P, P, P]),
        "useries_server_stats": (I, [P, P]),
        "useries_server_destroy": (I, [P]),
        "useries_server_hold": (I, [P, I]),
        "useries_philox4x32_10": (None, [P, P, P]),
        "useries_eval_static": (I, [P, I64, P, P, P, P, P, P]),
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


def useries_eval_static(plan, n, xyz, q, forces, energy, parts, stream=0):
    _check(lib().useries_eval_static(plan, int(n), xyz, q, forces, energy or None, parts or None,
                                     stream or None))


def useries_plan_info(plan):
    vals = [ctypes.c_double() for _ in range(5)]
    nt, ntg, nex, nsp = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    rk = (ctypes.c_int * 3)()
    eq33, f0, slope, ss, perr = (ctypes.c_double() for _ in range(5))
    P = ctypes.c_int()
    nc = (ctypes.c_int * 3)()
    _check(lib().useries_plan_info(plan, *[ctypes.byref(v) for v in vals], ctypes.byref(nt),
                                   ctypes.byref(eq33), ctypes.byref(f0), ctypes.byref(slope),
                                   ctypes.byref(ss), ctypes.byref(P), nc, ctypes.byref(perr),
                                   ctypes.byref(ntg), ctypes.byref(nex), ctypes.byref(nsp), rk))
    b, sigma, r0, w0, s0 = (v.value for v in vals)
    return dict(b=b, sigma=sigma, r0=r0, w0=w0, s0=s0, n_terms=nt.value, eq33=eq33.value,
                f_inf0=f0.value, c1_slope=slope.value, sigma_s=ss.value,
                stencil_half=P.value, ncell=tuple(nc), poly_maxerr=perr.value,
                n_terms_grid=ntg.value, near_exact=nex.value, n_terms_spectral=nsp.value,
                spectral_rank=tuple(rk))


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


def useries_server_default_opts():
    o = useries_server_opts()
    _check(lib().useries_server_default_opts(ctypes.byref(o)))
    return o


def useries_server_create(hbm_budget_bytes, max_slots, precision, opts=None):
    h = ctypes.c_void_p()
    _check(lib().useries_server_create(ctypes.byref(h), int(hbm_budget_bytes), int(max_slots),
                                       int(precision),
                                       ctypes.byref(opts) if opts is not None else None))
    return h.value


def useries_submit(server, req):
    """req: a useries_request; returns the ticket."""
    t = ctypes.c_uint64()
    _check(lib().useries_submit(server, ctypes.byref(req), ctypes.byref(t)))
    return t.value


def useries_poll(server, ticket):
    s = ctypes.c_int()
    _check(lib().useries_poll(server, ctypes.c_uint64(ticket), ctypes.byref(s)))
    return s.value


def useries_wait(server, ticket):
    s = ctypes.c_int()
    _check(lib().useries_wait(server, ctypes.c_uint64(ticket), ctypes.byref(s)))
    return s.value


def useries_request_times(server, ticket):
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().useries_request_times(server, ctypes.c_uint64(ticket), ctypes.byref(a),
                                       ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def useries_server_stats(server):
    out = (ctypes.c_int64 * 6)()
    _check(lib().useries_server_stats(server, out))
    keys = ("steps", "evals", "requests", "max_batch", "sum_batch", "graphs")
    return dict(zip(keys, (int(v) for v in out)))


def useries_server_hold(server, hold):
    _check(lib().useries_server_hold(server, int(bool(hold))))


def useries_server_destroy(server):
    _check(lib().useries_server_destroy(server))


def useries_philox4x32_10(counter, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xffffffff for v in counter])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    out = (ctypes.c_uint32 * 4)()
    lib().useries_philox4x32_10(c, k, out)
    return [int(v) for v in out]


def useries_strerror(code):
    return _strerror(code)


def useries_last_error():
    return lib().useries_last_error().decode()


__all__ = [n for n in dir() if n.startswith(("useries_", "USERIES_"))] + ["lib", "UseriesError"]
