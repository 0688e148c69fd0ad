"""GPU tests of the serving loop (useries_server_* / useries_submit / useries_poll).

* One evaluation of a request equals the one-box evaluation of the same cell
  (the batched launches run the same kernel bodies): bitwise.
* A request's results are the same alone and in a mix of other requests of
  uneven size, with graph replays and with eager launches, and when the HBM
  budget forces requests to wait for admission: bitwise, since no arithmetic
  of a box depends on the rest of the batch.
* A trajectory (evaluations with device-drawn displacements between them)
  matches the oracle at the positions of its last evaluation, and the
  displacements have the requested spread.
"""
import math

import numpy as np
import pytest

from gpu_util import log, oracle_eval, rel_rms

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_1911_01377_amd import (USERIES_BF16X3, USERIES_DONE, USERIES_PLAIN_FP32,  # noqa: E402
                                  Plan, Server, UseriesError, synth)
from paper_1911_01377_amd import _native as N  # noqa: E402

FORMS = [("plain", USERIES_PLAIN_FP32, 1e-6, 1e-5), ("bf16x3", USERIES_BF16X3, 1e-3, 1e-3)]


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def request_cell(k):
    """Request k of the serving stream: (xyz, q, box, r_c, grid) with grid
    spacing <= 1 A and r_c = min(9, 0.45 L)."""
    xyz, q, box = synth.serving_request(k)
    L = min(box)
    rc = min(9.0, 0.45 * L)
    grid = tuple(int(math.ceil(b)) for b in box)
    return xyz, q, box, rc, grid


def small_water(n_mol, seed):
    L = (n_mol / synth.WATER_DENSITY) ** (1.0 / 3.0)
    xyz, q, box = synth.water_box(n_mol=n_mol, L=L, seed=seed)
    return xyz, q, box, min(9.0, 0.45 * L), tuple(int(math.ceil(b)) for b in box)


def run_all(server, cells, n_evals, disp, seeds, want_positions=False):
    """Submit every cell while admissions are held, then release them together."""
    server.hold(True)
    tickets = [server.submit(x, q, box, rc, grid, n_evals=n_evals, disp_sigma=disp, seed=s,
                             want_positions=want_positions)
               for (x, q, box, rc, grid), s in zip(cells, seeds)]
    server.hold(False)
    return [server.result(t) for t in tickets]


@pytest.mark.parametrize("form,prec,e_tol,f_tol", FORMS)
def test_single_evaluation_equals_plan(form, prec, e_tol, f_tol):
    need_gpu()
    xyz, q, box, rc, grid = request_cell(3)
    log("case serve-vs-plan/%s: n=%d box=%.2f rc=%.2f grid=%s" % (form, len(q), box[0], rc, grid))
    srv = Server(256 << 20, max_slots=4, precision=prec)
    res = srv.result(srv.submit(xyz, q, box, rc, grid, n_evals=1))
    srv.close()
    plan = Plan(box, rc, grid, precision=prec)
    dev = torch.device("cuda:0")
    e, f, _ = plan.eval(torch.from_numpy(xyz).to(dev), torch.from_numpy(q).to(dev))
    torch.cuda.synchronize()
    e, f = float(e.cpu()[0]), f.cpu().numpy()
    plan.close()
    log("   E_server=%.15g E_plan=%.15g max|dF|=%.3e"
        % (res["energies"][0], e, float(np.max(np.abs(res["forces"] - f)))))
    assert res["energies"][0] == e
    assert np.array_equal(res["forces"], f)


def test_step_with_both_binning_sequences():
    """A flat 256 x 256 x 19 A cell of 200,000 random charges (69 x 69
    columns: more than the two-launch binning takes, so it bins in four
    launches) and a small water box (two-launch binning) admitted into the
    same steps: the step launches both sequences, each box's kernels take
    only their own, and each result equals the plan's evaluation bitwise."""
    need_gpu()
    big_xyz, big_q, big_box = synth.random_box(200000, (256.0, 256.0, 19.0), seed=31)
    cells = [(big_xyz, big_q, big_box, 9.0, (128, 128, 20)), small_water(216, 11)]
    log("case mixed-binning: sizes %s" % [len(c[1]) for c in cells])
    srv = Server(1 << 30, max_slots=4, precision=USERIES_BF16X3)
    res = run_all(srv, cells, 1, 0.0, [5, 6])
    st = srv.stats()
    srv.close()
    assert st["max_batch"] == 2, st
    dev = torch.device("cuda:0")
    for (xyz, q, box, rc, grid), r in zip(cells, res):
        plan = Plan(box, rc, grid, precision=USERIES_BF16X3)
        e, f, _ = plan.eval(torch.from_numpy(xyz).to(dev), torch.from_numpy(q).to(dev))
        torch.cuda.synchronize()
        e, f = float(e.cpu()[0]), f.cpu().numpy()
        ncell = N.useries_plan_info(plan.handle)["ncell"]   # the columns of this evaluation
        plan.close()
        log("   n=%d columns %s: E_server=%.15g E_plan=%.15g max|dF|=%.3e"
            % (len(q), ncell, r["energies"][0], e, float(np.max(np.abs(r["forces"] - f)))))
        assert r["energies"][0] == e
        assert np.array_equal(r["forces"], f)
        if len(q) == 200000:
            assert ncell[0] * ncell[1] > 4096, ncell


@pytest.mark.parametrize("form,prec,e_tol,f_tol", FORMS)
def test_alone_equals_mix(form, prec, e_tol, f_tol):
    need_gpu()
    cells = [request_cell(k) for k in (0, 1, 2, 5, 7)] + [small_water(216, 11)]
    seeds = [101 + 7 * k for k in range(len(cells))]
    log("case alone-vs-mix/%s: sizes %s" % (form, [len(c[1]) for c in cells]))
    n_evals, disp = 4, 0.02
    # alone: one request at a time on a fresh server
    alone = []
    for c, s in zip(cells, seeds):
        srv = Server(512 << 20, max_slots=8, precision=prec)
        alone.append(run_all(srv, [c], n_evals, disp, [s], want_positions=True)[0])
        srv.close()
    variants = [
        ("mix, graph", dict(budget=1 << 30, use_graph=1)),
        ("mix, eager launches", dict(budget=1 << 30, use_graph=0)),
        ("mix, small budget", dict(budget=16 << 20, use_graph=1)),
    ]
    for name, v in variants:
        srv = Server(v["budget"], max_slots=8, precision=prec, use_graph=v["use_graph"])
        mix = run_all(srv, cells, n_evals, disp, seeds, want_positions=True)
        st = srv.stats()
        srv.close()
        log("   %s: stats %s" % (name, st))
        assert st["requests"] == len(cells) and st["evals"] == len(cells) * n_evals
        if v["budget"] < (1 << 30):
            assert st["max_batch"] < len(cells)   # the budget made requests wait
        else:
            assert st["max_batch"] == len(cells)
        for k, (a, m) in enumerate(zip(alone, mix)):
            assert np.array_equal(a["energies"], m["energies"]), (name, k)
            assert np.array_equal(a["forces"], m["forces"]), (name, k)
            assert np.array_equal(a["xyz_final"], m["xyz_final"]), (name, k)


@pytest.mark.parametrize("form,prec,e_tol,f_tol", FORMS)
def test_trajectory_against_oracle(form, prec, e_tol, f_tol):
    need_gpu()
    xyz, q, box, rc, grid = small_water(216, 5)
    n_evals, disp = 5, 0.02
    log("case trajectory/%s: n=%d box=%.2f rc=%.2f grid=%s" % (form, len(q), box[0], rc, grid))
    srv = Server(256 << 20, max_slots=2, precision=prec)
    res = srv.result(srv.submit(xyz, q, box, rc, grid, n_evals=n_evals, disp_sigma=disp,
                                seed=77, want_positions=True))
    srv.close()
    plan = Plan(box, rc, grid, precision=prec)
    info = plan.info
    plan.close()
    # first evaluation: the input positions; last: the returned positions
    o0, _ = oracle_eval(xyz, q, box, info, rc)
    o1, f1 = oracle_eval(res["xyz_final"], q, box, info, rc)
    de0 = abs(res["energies"][0] - o0["total"]) / abs(o0["total"])
    de1 = abs(res["energies"][-1] - o1["total"]) / abs(o1["total"])
    df = rel_rms(res["forces"].astype(np.float64), f1)
    log("   dE(first)=%.2e dE(last)=%.2e dF(last)=%.2e energies=%s"
        % (de0, de1, df, np.array2string(res["energies"], precision=6)))
    assert de0 <= e_tol and de1 <= e_tol and df <= f_tol
    # displacements: n_evals - 1 moves of N(0, disp^2) per coordinate
    d = res["xyz_final"].astype(np.float64) - xyz.astype(np.float64)
    d -= np.round(d / np.array(box)) * np.array(box)
    want = disp * math.sqrt(n_evals - 1)
    log("   displacement mean %.3e std %.5f (want %.5f)" % (d.mean(), d.std(), want))
    assert abs(d.std() / want - 1.0) < 0.08
    assert abs(d.mean()) < 5.0 * want / math.sqrt(d.size)


def test_requests_that_cannot_fit_are_refused():
    need_gpu()
    xyz, q, box, rc, grid = request_cell(2)
    log("case refuse: n=%d" % len(q))
    srv = Server(4 << 20, max_slots=2, precision=USERIES_BF16X3)
    with pytest.raises(UseriesError) as e:
        srv.submit(xyz, q, box, rc, grid)
    assert e.value.code == N.USERIES_ENOMEM
    with pytest.raises(UseriesError) as e:
        srv.submit(xyz, q, box, 0.6 * min(box), grid)   # r_c beyond L/2
    assert e.value.code == N.USERIES_EINVAL
    srv.close()


def test_poll_states():
    need_gpu()
    cells = [small_water(216, 21), small_water(400, 22)]
    log("case poll: sizes %s" % [len(c[1]) for c in cells])
    srv = Server(256 << 20, max_slots=1, precision=USERIES_BF16X3)
    t = [srv.submit(x, q, box, rc, grid, n_evals=3, disp_sigma=0.02, seed=k)
         for k, (x, q, box, rc, grid) in enumerate(cells)]
    assert srv.poll(t[0]) in (N.USERIES_PENDING, N.USERIES_RUNNING, USERIES_DONE)
    for tk in t:
        assert srv.wait(tk) == USERIES_DONE
        ts, ta, td = srv.times(tk)
        assert 0 <= ts <= ta <= td
    # one slot: the second request was admitted after the first one finished
    assert srv.times(t[1])[1] >= srv.times(t[0])[2] - 1e-3
    with pytest.raises(UseriesError) as e:
        N.useries_poll(srv.handle, 987654321)
    assert e.value.code == N.USERIES_ENOTFOUND
    srv.close()
