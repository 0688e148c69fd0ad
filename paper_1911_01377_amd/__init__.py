"""u-series electrostatics on MI355X (gfx950).

The computation lives in the HIP library ``libuseries.so`` behind the C ABI of
``include/useries.h``; :mod:`paper_1911_01377_amd._native` binds it with the
same names.  :class:`Plan` is a small convenience wrapper over PyTorch device
tensors (PyTorch provides device memory and streams only).
"""
from . import _native
from ._native import (USERIES_C0, USERIES_C1, USERIES_C2_B2, USERIES_TABLE1_ROW1,
                      USERIES_TABLE1_ROW2, USERIES_TABLE1_ROW3, USERIES_PLAIN_FP32,
                      USERIES_BF16X3, UseriesError)

__all__ = ["Plan", "UseriesError", "USERIES_C0", "USERIES_C1", "USERIES_C2_B2",
           "USERIES_TABLE1_ROW1", "USERIES_TABLE1_ROW2", "USERIES_TABLE1_ROW3",
           "USERIES_PLAIN_FP32", "USERIES_BF16X3"]


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
