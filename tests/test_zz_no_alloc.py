"""The scratch-free EM entry point (ctis_em_iterate_static, the library's
static device array in place of the workspace) against ctis_em_iterate on the
same inputs: bit for bit, on two calls in a row with the second on a smaller
frame, and the size limit."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2006_01573_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a visible MI355X"
    return _t


@pytest.fixture(scope="module")
def ctis(torch):
    from paper_2006_01573_amd import ctis as _c
    _c.load_library()
    return _c


def frame(torch, plan, case):
    g = plan.forward(torch.from_numpy(case.f_true.astype(np.float32)).cuda())
    return torch.from_numpy(case.noisy(g.double().cpu().numpy())).cuda()


def static_call(torch, ctis, plan, g, f, iters):
    """ctis_em_iterate_static through the C ABI, on the current stream."""
    L = ctis.load_library()
    st = L.ctis_em_iterate_static(plan._handle, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                  int(iters), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def test_static_scratch_matches_workspace_call(torch, ctis):
    """c2 (20 iterations), then the smaller c1 frame (7 iterations): each equals
    ctis_em_iterate with a workspace of its own, bit for bit."""
    for cfg, iters in ((2, 20), (1, 7)):
        case = W.make_case(cfg)
        plan = ctis.Plan.from_case(case)
        assert plan.info.workspace_bytes <= 16 << 20
        g = frame(torch, plan, case)
        log(f"static scratch: c{cfg}, {iters} iterations, region path {plan.info.em_region_path}")
        ref = plan.em(g, iters)
        f = torch.ones(plan.shape_f, device="cuda")
        assert static_call(torch, ctis, plan, g, f, iters) == 0
        torch.cuda.synchronize()
        assert torch.equal(f, ref)
        # the binding's wrapper takes the same route
        f2 = plan.em_static(g, iters, torch.ones(plan.shape_f, device="cuda"))
        assert torch.equal(f2, ref)
        plan.close()


def test_static_scratch_size_limit(torch, ctis):
    """A plan whose EM workspace exceeds the static array is refused before
    any launch."""
    geo = W.Geometry(4, 4, 1, 2048, 2048)            # u alone is 16 MiB
    ptr, idx, val = W.random_kernels(geo, 3, np.random.default_rng(1))
    plan = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)
    assert plan.info.workspace_bytes > 16 << 20
    g = torch.ones(plan.shape_g, device="cuda")
    f = torch.ones(plan.shape_f, device="cuda")
    st = static_call(torch, ctis, plan, g, f, 1)
    assert ctis.STATUS_NAMES[st] == "CTIS_E_TOO_LARGE"
    assert torch.equal(f, torch.ones_like(f))
    plan.close()
