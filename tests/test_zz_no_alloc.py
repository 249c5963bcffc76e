"""pmdg_bind_static, the entry point for callers that cannot allocate: the
solver's workspace is the library's static per-device array instead of a
caller buffer.  Two binds in a row, the second with a smaller problem, each
give bitwise the traces and state of the same solver bound to caller memory
(same kernels); the first solver is refused once the second has taken the
array; a problem beyond the array's size is refused."""
import numpy as np
import pytest

from paper_2603_06267_amd import _lib, solver, workloads as W

pytestmark = pytest.mark.gpu


def _run(wl, precision, steps, bind):
    g = solver.from_workload(wl, precision=precision, n_steps=steps, shape_fn=W.shape_fn(wl), bind=bind)
    g.step(steps)
    return g, g.read_traces(), g.get_state(0), g.read_modal(0)


def _same(a, b):
    for x, y in zip(a[1:], b[1:]):
        if isinstance(x, tuple):
            for u, v in zip(x, y):
                assert np.array_equal(u, v)
        else:
            assert np.array_equal(x, y)


def test_bind_static_two_calls():
    steps = 120
    big = W.small_two_domain(False, steps=steps)     # 4:3 two-domain case, 0.9 MiB
    small = W.config1()                               # cube, 0.4 MiB
    print("bind_static: 4:3 two-domain FP32, then cube FP64", flush=True)
    a_static = _run(big, 32, steps, "static")
    a_caller = _run(big, 32, steps, True)
    _same(a_static, a_caller)
    assert np.abs(a_static[1]).max() > 0
    b_static = _run(small, 64, steps, "static")
    b_caller = _run(small, 64, steps, True)
    _same(b_static, b_caller)
    # the first solver's workspace now belongs to the second
    with pytest.raises(_lib.PmdgError) as e:
        a_static[0].step(1)
    assert e.value.code == _lib.PMDG_ESTATE
    with pytest.raises(_lib.PmdgError) as e:
        a_static[0].read_traces()
    assert e.value.code == _lib.PMDG_ESTATE
    # after the owner is destroyed the array can be bound again
    b_static[0].close()
    c_static = _run(small, 32, 40, "static")
    c_caller = _run(small, 32, 40, True)
    _same(c_static, c_caller)
    c_static[0].close()


def test_bind_static_rejects_oversized_problem():
    wl = W.config2()
    g = solver.from_workload(wl, precision=64, n_steps=100, scenarios=[0] * 8, shape_fn=W.shape_fn(wl),
                             bind=False)
    assert g.workspace_size() > 32 << 20
    with pytest.raises(_lib.PmdgError) as e:
        g.bind_static()
    assert e.value.code == _lib.PMDG_ENOMEM
