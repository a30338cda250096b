"""heom_propagate_noalloc: the propagation entry point that allocates
nothing (its work vectors live in the library's static device array). Called
through the C ABI, it must equal heom_propagate with a caller work buffer --
bitwise, since both run the same kernels -- on two calls in a row, the second
with a smaller state (the array keeps the first call's contents), and refuse
tables whose work memory exceeds HEOM_NOALLOC_WORK_BYTES."""
import numpy as np
import pytest

from paper_2608_20657_amd import workloads as W
from tests.gpu_util import gpu_propagate, named_tier0, torch_cuda, upload

pytestmark = pytest.mark.gpu


def noalloc_run(T, torch, tier0, dt, steps, every, precision):
    info = T.info()
    s = torch.cuda.current_stream()
    y = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
    T.init_state(tier0, y, s)
    nobs = steps // every + 1 if every > 0 else 0
    obs = torch.zeros(max(nobs, 1) * 10, dtype=torch.float64, device="cuda")
    T.propagate_noalloc(y, dt, steps, every, obs if every > 0 else None, precision, s)
    torch.cuda.synchronize()
    return y.cpu().numpy(), obs.cpu().numpy().reshape(-1, 10)[:nobs]


@pytest.mark.parametrize("precision", [0, 1, 2, 3])
def test_noalloc_equals_caller_buffer(precision):
    from paper_2608_20657_amd import heom
    torch = torch_cuda()
    # first a larger state (the saturated workload, 263,583 variables; compact
    # tiles when the Hermitian flag is set), then a smaller one (21,105)
    cases = [(W.config_saturated(), "upper_polariton", 30, 10), (W.config_localized(), "site1", 50, 10)]
    for p, state, steps, every in cases:
        T, _ = upload(p)
        if precision & heom.HEOM_HERMITIAN:
            T.set_tuning(compact=1)
            img = torch.empty(T.info()["table_bytes"], dtype=torch.uint8, device="cuda")
            T.upload(img, torch.cuda.current_stream())
        assert T.info()["work_bytes_fp64"] <= heom.HEOM_NOALLOC_WORK_BYTES
        t0 = named_tier0(T, p, state)
        ya, oa = noalloc_run(T, torch, t0, 0.02, steps, every, precision)
        yb, ob = gpu_propagate(T, torch, t0, 0.02, steps, every, precision)
        assert np.array_equal(ya.view(np.float64), yb.view(np.float64)), p.N
        assert np.array_equal(oa, ob), p.N
        assert np.isfinite(ya).all() and np.abs(ya).max() > 0


def test_noalloc_refuses_too_large_tables():
    from paper_2608_20657_amd import heom
    p = W.random_problem(100, 4, 8, 0, seed=3)       # 1.56 M variables, transposed copies: 125 MB of work
    T, torch = upload(p)
    assert T.info()["work_bytes_fp64"] > heom.HEOM_NOALLOC_WORK_BYTES
    y = torch.zeros(T.info()["n_var"], dtype=torch.complex128, device="cuda")
    with pytest.raises(heom.HeomError) as e:
        T.propagate_noalloc(y, 0.02, 1, 0, None, 0, torch.cuda.current_stream())
    assert e.value.code == -3
