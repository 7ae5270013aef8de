"""The allocation-free entry point nedner_corrcoef_noalloc (partial sums in
the library's file-scope device scratch) against nedner_corrcoef (partial
sums in a caller workspace): two calls in a row, the second on a smaller
input and another dtype, each equal bit for bit to the workspace entry
point's result (the same kernels add the same terms in the same order) and
to the oracle's coefficient. Calls go through the C-ABI."""
import ctypes

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _call(torch, L, fn_name, a, b, mask, dtype_code):
    res = torch.full((1,), float("nan"), dtype=torch.float64, device=a.device)
    stream = ctypes.c_void_p(torch.cuda.current_stream(a.device).cuda_stream)
    mp = ctypes.c_void_p(mask.data_ptr()) if mask is not None else ctypes.c_void_p(0)
    if fn_name == "nedner_corrcoef":
        work = torch.empty(int(L.nedner_metrics_workspace_size()), dtype=torch.uint8, device=a.device)
        st = L.nedner_corrcoef(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), mp, a.numel(),
                               dtype_code, ctypes.c_void_p(res.data_ptr()), ctypes.c_void_p(work.data_ptr()),
                               work.numel(), stream)
    else:
        st = L.nedner_corrcoef_noalloc(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), mp,
                                       a.numel(), dtype_code, ctypes.c_void_p(res.data_ptr()), stream)
    assert st == 0, L.nedner_last_error()
    torch.cuda.synchronize()
    return float(res.item())


def test_noalloc_matches_workspace_entry_point(torch_gpu):
    import paper_1501_02946_amd as N
    torch = torch_gpu
    L = N.lib()
    rng = np.random.default_rng(42)
    cases = [
        # first call: a large float32 input with a mask
        (np.float32, 3_000_001, True, 0),
        # second call, smaller, float64, no mask: nothing of the first call's
        # partial sums may leak into it
        (np.float64, 1537, False, 1),
    ]
    for dt, n, use_mask, code in cases:
        a = rng.normal(size=n).astype(dt)
        b = (0.4 * a + rng.normal(size=n)).astype(dt)
        m = rng.random(n) < 0.7 if use_mask else None
        ta = torch.as_tensor(a, device="cuda")
        tb = torch.as_tensor(b, device="cuda")
        tm = torch.as_tensor(m.astype(np.uint8), device="cuda") if use_mask else None
        print(f"corrcoef_noalloc: n={n} dtype={np.dtype(dt).name} mask={use_mask}", flush=True)
        want = _call(torch, L, "nedner_corrcoef", ta, tb, tm, code)
        got = _call(torch, L, "nedner_corrcoef_noalloc", ta, tb, tm, code)
        assert got == want, (got, want)
        ref = O.corrcoef(a, b, m)
        assert abs(got - ref) <= 1e-12 * abs(ref), (got, ref)
    # and again on the first input after the smaller one
    a = rng.normal(size=10_000).astype(np.float32)
    ta = torch.as_tensor(a, device="cuda")
    tb = torch.as_tensor((a * a).astype(np.float32), device="cuda")
    assert _call(torch, L, "nedner_corrcoef_noalloc", ta, tb, None, 0) == \
        _call(torch, L, "nedner_corrcoef", ta, tb, None, 0)


def test_noalloc_argument_errors(torch_gpu):
    import paper_1501_02946_amd as N
    L = N.lib()
    assert L.nedner_corrcoef_noalloc(None, None, None, 4, 0, None, None) == 1
    torch = torch_gpu
    x = torch.ones(8, device="cuda")
    r = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert L.nedner_corrcoef_noalloc(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), None, 0, 0,
                                     ctypes.c_void_p(r.data_ptr()), None) == 1
    assert L.nedner_corrcoef_noalloc(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), None, 8, 7,
                                     ctypes.c_void_p(r.data_ptr()), None) == 1
