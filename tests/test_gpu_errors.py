"""Error paths of a live plan, forced from the host (nothing here launches a
kernel that could fail, and no kernel is made to fault):

* NEDNER_E_WORKSPACE: an execute before any workspace is set, and a workspace
  smaller than nedner_workspace_size, are refused before any launch;
* NEDNER_E_STATE: after a HIP error (injected by nedner_debug_inject_hip_error,
  which puts the plan into the state a failed HIP call leaves) every execute,
  tuning and profiling call is refused, and nedner_destroy still works.
"""
import ctypes

import numpy as np
import pytest

import synth
from gpu_util import make_plan, to_dev

pytestmark = pytest.mark.gpu
E_HIP, E_STATE, E_WORKSPACE, OK = 5, 7, 4, 0


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def test_workspace_errors(torch_gpu):
    import paper_1501_02946_amd as N
    torch = torch_gpu
    L = N.lib()
    p = synth.config("c5sub")
    plan = make_plan(p, "fp32c")
    g = to_dev(p.g, plan)
    out = torch.zeros((p.n1, p.n2, p.n3), dtype=plan.dtype, device=plan.device)
    stream = plan._stream()
    # no workspace yet: refused, output untouched
    assert L.nedner_execute(plan._plan, _ptr(g), _ptr(out), 0, stream) == E_WORKSPACE
    assert L.nedner_execute_adjoint(plan._plan, _ptr(out), 0, _ptr(g), stream) == E_WORKSPACE
    assert b"workspace" in L.nedner_last_error()
    need = ctypes.c_size_t(0)
    assert L.nedner_workspace_size(plan._plan, ctypes.byref(need)) == OK
    small = torch.empty(max(need.value // 2, 256), dtype=torch.uint8, device=plan.device)
    assert L.nedner_set_workspace(plan._plan, _ptr(small), ctypes.c_size_t(small.numel())) == E_WORKSPACE
    assert L.nedner_execute(plan._plan, _ptr(g), _ptr(out), 0, stream) == E_WORKSPACE
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0
    # with the workspace the same call runs
    vol = plan(g)
    torch.cuda.synchronize()
    assert np.isfinite(vol.cpu().numpy()).all()


def test_state_after_injected_hip_error(torch_gpu):
    import paper_1501_02946_amd as N
    torch = torch_gpu
    L = N.lib()
    p = synth.config("c5sub")
    plan = make_plan(p, "fp64")
    g = to_dev(p.g, plan)
    ref = plan(g).cpu().numpy()
    out = torch.zeros_like(plan(g))
    stream = plan._stream()
    # hipErrorLaunchFailure (719) as a failing HIP call would have returned it
    assert L.nedner_debug_inject_hip_error(plan._plan, 719) == E_HIP
    assert b"injected" in L.nedner_last_error()
    assert L.nedner_execute(plan._plan, _ptr(g), _ptr(out), 0, stream) == E_STATE
    assert L.nedner_execute_adjoint(plan._plan, _ptr(out), 0, _ptr(g), stream) == E_STATE
    assert L.nedner_execute_q(plan._plan, _ptr(out), _ptr(g), stream) == E_STATE
    assert L.nedner_profile_begin(plan._plan, 4) == E_STATE
    t = N.tuning_struct()
    assert L.nedner_get_tuning(plan._plan, ctypes.byref(t)) == OK
    assert L.nedner_set_tuning(plan._plan, ctypes.byref(t)) == E_STATE
    assert L.nedner_autotune(plan._plan, _ptr(g), stream, ctypes.byref(t)) == E_STATE
    with pytest.raises(N.NednerError):
        plan(g)
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0
    plan.close()
    # a new plan on the same device is unaffected
    plan2 = make_plan(p, "fp64")
    assert np.array_equal(plan2(to_dev(p.g, plan2)).cpu().numpy(), ref)
