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


def oracle_params(info, rc):
    return oracle.Params(b=info["b"], sigma=info["sigma"], w0=info["w0"], s0=info["s0"], rc=rc,
                         nterms=info["n_terms"])


def oracle_eval(xyz, q, box, info, rc):
    p = oracle_params(info, rc)
    parts, f = oracle.eval_full(np.asarray(xyz, np.float64), np.asarray(q, np.float64), box, p)
    return parts, f


def rel_rms(f, g):
    den = np.sum(g ** 2)
    return math.sqrt(np.sum((f - g) ** 2) / den) if den > 0 else math.sqrt(np.sum(f ** 2))


def compare(tag, xyz, q, box, rc, grid, e_tol, f_tol, **kw):
    log("case %s: n=%d box=%s rc=%g grid=%s %s" % (tag, len(q), tuple(box), rc, tuple(grid), kw))
    gparts, gf, info = gpu_eval(xyz, q, box, rc, grid, **kw)
    oparts, of = oracle_eval(xyz, q, box, info, rc)
    de = abs(gparts[4] - oparts["total"]) / max(abs(oparts["total"]), 1e-300)
    df = rel_rms(gf, of)
    log("   E_gpu=%.12g E_oracle=%.12g dE=%.2e dF=%.2e" % (gparts[4], oparts["total"], de, df))
    for k, name in enumerate(("near", "far", "self", "bg")):
        log("   %-4s gpu=%.15g oracle=%.15g diff=%.3e"
            % (name, gparts[k], oparts[name], gparts[k] - oparts[name]))
    assert de <= e_tol, (tag, de)
    assert df <= f_tol, (tag, df)
    return gparts, gf, oparts, of, info
