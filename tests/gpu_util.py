"""Helpers shared by the GPU parity tests: run the library through the C ABI
and the FP64 oracle on the same float32 inputs, and compare."""
import math
import sys

import numpy as np

import oracle


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_eval(xyz, q, box, rc, grid, **kw):
    """(parts[5] float64, forces [n,3] float64, plan info) from the HIP library."""
    import torch
    from paper_1911_01377_amd import Plan
    plan = Plan(box, rc, grid, **kw)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(np.ascontiguousarray(xyz, dtype=np.float32)).to(dev)
    qq = torch.from_numpy(np.ascontiguousarray(q, dtype=np.float32)).to(dev)
    parts = torch.zeros(5, dtype=torch.float64, device=dev)
    energy, forces, _ = plan.eval(x, qq, parts=parts)
    torch.cuda.synchronize()
    from paper_1911_01377_amd import _native
    info = _native.useries_plan_info(plan.handle)   # after the evaluation: its column grid
    out = parts.cpu().numpy().copy(), forces.cpu().numpy().astype(np.float64), info
    assert abs(float(energy.cpu()[0]) - out[0][4]) == 0.0
    plan.close()
    return out


def oracle_params(info, rc, alpha=1):
    return oracle.Params(b=info["b"], sigma=info["sigma"], w0=info["w0"], s0=info["s0"], rc=rc,
                         nterms=info["n_terms"], alpha=float(alpha))


def oracle_eval(xyz, q, box, info, rc, alpha=1):
    p = oracle_params(info, rc, alpha)
    parts, f = oracle.eval_full(np.asarray(xyz, np.float64), np.asarray(q, np.float64), box, p)
    return parts, f


def rel_rms(f, g):
    den = np.sum(g ** 2)
    return math.sqrt(np.sum((f - g) ** 2) / den) if den > 0 else math.sqrt(np.sum(f ** 2))


def max_atom_err(f, g):
    """Largest per-charge force error, each relative to the larger of that
    charge's reference force and the RMS reference force; returns (error,
    index, |F_ref| / rms of that charge)."""
    if len(g) == 0:
        return 0.0, -1, 0.0
    rms = math.sqrt(np.mean(np.sum(g ** 2, axis=1)))
    mag = np.sqrt(np.sum(g ** 2, axis=1))
    if rms == 0.0:    # forces that vanish by symmetry (one charge): absolute errors
        err = np.sqrt(np.sum((f - g) ** 2, axis=1))
        k = int(np.argmax(err))
        return float(err[k]), k, 0.0
    err = np.sqrt(np.sum((f - g) ** 2, axis=1)) / np.maximum(mag, rms)
    k = int(np.argmax(err))
    return float(err[k]), k, float(mag[k] / rms) if rms > 0 else 0.0


# A single charge may err by at most this multiple of the RMS force tolerance,
# relative to its own force or, for charges with less than the RMS force, to
# the RMS force: an error confined to a few charges (a mis-binned charge at a
# column or brick edge) does not show in the RMS.  (Random charges have a
# heavy-tailed force distribution, close pairs with forces far above the
# RMS, whose FP32 error is relative to their own force.)
ATOM_FACTOR = 10.0


def compare(tag, xyz, q, box, rc, grid, e_tol, f_tol, e_scale="total", **kw):
    """GPU vs oracle on the same inputs.  The energy error is relative to
    |E_total| (e_scale="total"), or, for random charges whose total is a
    small difference of much larger parts, to |E_near| + |E_far| + |E_self|
    (e_scale="parts"): each part carries its own rounding, relative to its
    own size, whatever the cancellation between them."""
    log("case %s: n=%d box=%s rc=%g grid=%s %s" % (tag, len(q), tuple(box), rc, tuple(grid), kw))
    gparts, gf, info = gpu_eval(xyz, q, box, rc, grid, **kw)
    oparts, of = oracle_eval(xyz, q, box, info, rc, kw.get("alpha", 1))
    if e_scale == "parts":
        escale = abs(oparts["near"]) + abs(oparts["far"]) + abs(oparts["self"])
    else:
        escale = abs(oparts["total"])
    de = abs(gparts[4] - oparts["total"]) / max(escale, 1e-300)
    df = rel_rms(gf, of)
    da, ka, ma = max_atom_err(gf, of)
    log("   E_gpu=%.12g E_oracle=%.12g dE=%.2e (vs %s) dF=%.2e max_i|dF_i|/max(|F_i|,rms)=%.2e "
        "(charge %d, |F|=%.2f rms) (N=%d, exact near terms %d)"
        % (gparts[4], oparts["total"], de, e_scale, df, da, ka, ma, info["n_terms"],
           info["near_exact"]))
    for k, name in enumerate(("near", "far", "self", "bg")):
        log("   %-4s gpu=%.15g oracle=%.15g diff=%.3e"
            % (name, gparts[k], oparts[name], gparts[k] - oparts[name]))
    assert de <= e_tol, (tag, de)
    assert df <= f_tol, (tag, df)
    assert da <= ATOM_FACTOR * f_tol, (tag, da)
    return gparts, gf, oparts, of, info
