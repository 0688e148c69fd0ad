"""u-series electrostatics on MI355X (gfx950).

The computation lives in the HIP library ``libuseries.so`` behind the C ABI of
``include/useries.h``; :mod:`paper_1911_01377_amd._native` binds it with the
same names.  :class:`Plan` is a small convenience wrapper over PyTorch device
tensors (PyTorch provides device memory and streams only).
"""
from . import _native
from ._native import (USERIES_C0, USERIES_C1, USERIES_C2_B2, USERIES_TABLE1_ROW1,
                      USERIES_TABLE1_ROW2, USERIES_TABLE1_ROW3, USERIES_PLAIN_FP32,
                      USERIES_BF16X3, USERIES_PENDING, USERIES_RUNNING, USERIES_DONE,
                      USERIES_ERROR, UseriesError)

__all__ = ["Plan", "Server", "UseriesError", "USERIES_C0", "USERIES_C1", "USERIES_C2_B2",
           "USERIES_TABLE1_ROW1", "USERIES_TABLE1_ROW2", "USERIES_TABLE1_ROW3",
           "USERIES_PLAIN_FP32", "USERIES_BF16X3", "USERIES_PENDING", "USERIES_RUNNING",
           "USERIES_DONE", "USERIES_ERROR"]


class Plan:
    """A u-series plan for one cell shape.

    Plan(box, r_c, grid, b=2.0, sigma=0.0, n_terms=0, construction=USERIES_C1,
         precision=USERIES_PLAIN_FP32, **opts)
    ``opts`` may set sigma_s_over_h, stencil_half, nterms_tol, poly_degree,
    max_atoms (see useries_opts).
    """

    def __init__(self, box, r_c, grid, b=2.0, sigma=0.0, n_terms=0, construction=USERIES_C1,
                 precision=USERIES_PLAIN_FP32, **opts):
        o = _native.useries_default_opts()
        o.construction = construction
        o.precision = precision
        for k, v in opts.items():
            if not hasattr(o, k):
                raise TypeError("unknown option %s" % k)
            setattr(o, k, v)
        self.box = tuple(float(v) for v in box)
        self.grid = tuple(int(v) for v in grid)
        self.handle = _native.useries_plan(self.box, r_c, b, sigma, n_terms, self.grid, o)
        self.info = _native.useries_plan_info(self.handle)

    def eval(self, xyz, q, forces=None, energy=None, parts=None, stream=None):
        """Asynchronous evaluation on ``stream`` (default: torch's current stream).
        xyz: float32 [n, 3] cuda tensor, q: float32 [n]; returns (energy[1] float64,
        forces [n, 3] float32, parts[5] float64 or None)."""
        import torch
        n = int(q.shape[0])
        if xyz.dtype != torch.float32 or q.dtype != torch.float32:
            raise TypeError("xyz and q must be float32")
        if not (xyz.is_cuda and q.is_cuda):
            raise TypeError("xyz and q must be device tensors")
        if tuple(xyz.shape) != (n, 3) or not xyz.is_contiguous() or not q.is_contiguous():
            raise ValueError("xyz must be contiguous [n, 3] and q contiguous [n]")
        dev = xyz.device
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float32, device=dev)
        if energy is None:
            energy = torch.empty(1, dtype=torch.float64, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev).cuda_stream
        if parts is not None:
            _native.useries_eval_parts(self.handle, n, xyz.data_ptr(), q.data_ptr(),
                                       forces.data_ptr(), energy.data_ptr(), parts.data_ptr(),
                                       stream)
        else:
            _native.useries_eval(self.handle, n, xyz.data_ptr(), q.data_ptr(),
                                 forces.data_ptr(), energy.data_ptr(), stream)
        return energy, forces, parts

    def timing(self, enable=None):
        if enable is not None:
            _native.useries_timing_enable(self.handle, enable)
            return None
        return _native.useries_timing_read(self.handle)

    def close(self):
        if self.handle:
            _native.useries_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server of independent cells (useries_server_* of the C ABI).

    Server(hbm_budget_bytes, max_slots=32, precision=USERIES_BF16X3, **opts)
    ``opts`` may set construction, b, nterms_tol, poly_degree, use_graph, inflight.
    The host arrays of a request are kept alive here until it is collected.
    """

    def __init__(self, hbm_budget_bytes, max_slots=32, precision=USERIES_BF16X3, **opts):
        o = _native.useries_server_default_opts()
        for k, v in opts.items():
            if not hasattr(o, k):
                raise TypeError("unknown option %s" % k)
            setattr(o, k, v)
        self.handle = _native.useries_server_create(hbm_budget_bytes, max_slots, precision, o)
        self._live = {}

    def submit(self, xyz, q, box, r_c, grid, n_evals=1, disp_sigma=0.0, seed=0,
               want_positions=False):
        """Queue one request; returns its ticket.  xyz float32 [n, 3], q float32 [n]
        (host arrays)."""
        import numpy as np
        xyz = np.ascontiguousarray(xyz, dtype=np.float32)
        q = np.ascontiguousarray(q, dtype=np.float32)
        n = int(q.shape[0])
        if xyz.shape != (n, 3):
            raise ValueError("xyz must be [n, 3]")
        energies = np.zeros(int(n_evals), dtype=np.float64)
        forces = np.zeros((n, 3), dtype=np.float32)
        xyz_final = np.zeros((n, 3), dtype=np.float32) if want_positions else None
        r = _native.useries_request()
        r.n = n
        r.xyz = xyz.ctypes.data
        r.q = q.ctypes.data
        for a in range(3):
            r.box[a] = float(box[a])
            r.grid[a] = int(grid[a])
        r.r_c = float(r_c)
        r.n_evals = int(n_evals)
        r.disp_sigma = float(disp_sigma)
        r.seed = int(seed) & 0xffffffffffffffff
        r.energies = energies.ctypes.data
        r.forces = forces.ctypes.data
        r.xyz_final = xyz_final.ctypes.data if xyz_final is not None else None
        t = _native.useries_submit(self.handle, r)
        self._live[t] = (xyz, q, energies, forces, xyz_final)
        return t

    def poll(self, ticket):
        return _native.useries_poll(self.handle, ticket)

    def wait(self, ticket):
        return _native.useries_wait(self.handle, ticket)

    def result(self, ticket):
        """Wait for the ticket; returns dict(energies, forces, xyz_final, times) and
        releases the host arrays held for it.  Raises UseriesError if it failed."""
        st = _native.useries_wait(self.handle, ticket)
        _, _, energies, forces, xyz_final = self._live.pop(ticket)
        if st != USERIES_DONE:
            raise UseriesError(_native.USERIES_EHIP, _native.useries_last_error())
        return dict(energies=energies, forces=forces, xyz_final=xyz_final,
                    times=_native.useries_request_times(self.handle, ticket))

    def times(self, ticket):
        return _native.useries_request_times(self.handle, ticket)

    def stats(self):
        return _native.useries_server_stats(self.handle)

    def hold(self, hold=True):
        """Pause (True) or resume (False) admissions."""
        _native.useries_server_hold(self.handle, hold)

    def close(self):
        if self.handle:
            _native.useries_server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
