"""useries_eval_static: the evaluation with its per-charge workspace in the
library's fixed device array (no allocation in the call), against
useries_eval_parts on the same plan and inputs.  The kernels and their
arithmetic are the same, so the outputs must agree bitwise, on two calls in
a row (the second with fewer charges, so that the array holds the first
call's larger layout) and in both precision forms."""
import numpy as np
import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_1911_01377_amd import USERIES_BF16X3, UseriesError, Plan, _native, synth  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _static(plan, x, q):
    n = q.shape[0]
    dev = x.device
    forces = torch.full((n, 3), float("nan"), dtype=torch.float32, device=dev)
    parts = torch.full((5,), float("nan"), dtype=torch.float64, device=dev)
    energy = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    _native.useries_eval_static(plan.handle, n, x.data_ptr(), q.data_ptr(), forces.data_ptr(),
                                energy.data_ptr(), parts.data_ptr(), stream)
    torch.cuda.synchronize()
    return energy.cpu().numpy(), parts.cpu().numpy(), forces.cpu().numpy()


def _eval(plan, x, q):
    parts = torch.zeros(5, dtype=torch.float64, device=x.device)
    energy, forces, _ = plan.eval(x, q, parts=parts)
    torch.cuda.synchronize()
    return energy.cpu().numpy(), parts.cpu().numpy(), forces.cpu().numpy()


@pytest.mark.parametrize("precision", [0, USERIES_BF16X3])
def test_static_workspace_matches_eval(precision):
    n_mol = 2000
    L = (n_mol / synth.WATER_DENSITY) ** (1 / 3)
    xyz, q, box = synth.water_box(n_mol=n_mol, L=L, seed=91)
    g = int(np.ceil(L))
    dev = torch.device("cuda:0")
    plan = Plan(box, 9.0, (g, g, g), precision=precision)
    try:
        # the second call has fewer charges (the first 1,300 molecules)
        for n in (len(q), 3 * 1300):
            log("case static workspace: precision=%d n=%d grid=%d" % (precision, n, g))
            x = torch.from_numpy(np.ascontiguousarray(xyz[:n])).to(dev)
            qq = torch.from_numpy(np.ascontiguousarray(q[:n])).to(dev)
            e_s, p_s, f_s = _static(plan, x, qq)
            e_r, p_r, f_r = _eval(plan, x, qq)
            log("   E static %.15g, E eval %.15g" % (e_s[0], e_r[0]))
            assert np.array_equal(p_s, p_r) and e_s[0] == p_r[4] and e_r[0] == p_r[4]
            assert np.array_equal(f_s, f_r)
    finally:
        plan.close()


def test_static_workspace_rejects_too_many_charges():
    """A charge count whose workspace exceeds the fixed array fails with
    USERIES_EINVAL before anything is launched."""
    dev = torch.device("cuda:0")
    plan = Plan((200.0, 200.0, 200.0), 9.0, (100, 100, 100))
    dummy = torch.zeros(4, dtype=torch.float32, device=dev)
    try:
        with pytest.raises(UseriesError) as ei:
            _native.useries_eval_static(plan.handle, 1_000_000, dummy.data_ptr(), dummy.data_ptr(),
                                        dummy.data_ptr(), 0, dummy.data_ptr(), 0)
        assert ei.value.code == _native.USERIES_EINVAL
        assert "fixed" in str(ei.value)
    finally:
        plan.close()
