"""qmc_integrate_static: the integration entry point that allocates no device memory
(its device state lives in the library's static scratch) against qmc_integrate on a
bound workspace, two calls in a row with the second on a smaller input, and against the
oracle on the smaller input's sums."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _pair(prob, **kw):
    import paper_2305_19768_amd as qmc
    ref = qmc.Plan(prob, **kw)
    st = qmc.Plan(prob, bind_workspace=False, **kw)
    assert st.workspace is None
    return ref, st


def _compare(ref, st):
    import torch
    q0, m0, e0 = ref.integrate()
    q1, m1, e1 = st.integrate_static()
    torch.cuda.synchronize()
    # same kernels, same reduction order: the sums agree bit for bit
    assert torch.equal(q0, q1)
    assert torch.equal(m0, m1) and torch.equal(e0, e1)
    return q1.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
def test_static_entry_point_matches_workspace_entry_point(precision):
    import oracle
    print(f"static scratch: two-loop 10 sectors then 3 sectors, precision {precision}", flush=True)
    big = W.two_loop_integral(seed=4, n_sectors=10, n_scale=0.03, m=16)
    small = W.two_loop_integral(seed=5, n_sectors=3, n_scale=0.003, m=8)
    _compare(*_pair(big, precision=precision))
    q = _compare(*_pair(small, precision=precision))   # the second call, smaller input
    tol = 1e-12 if precision == 0 else 1e-5
    for s, sec in enumerate(small.sectors):
        Qo, So = oracle.sector_sums(sec, small.shifts[s])
        bad = np.abs(q[s] - Qo) > tol * np.maximum(np.abs(Qo), So)
        assert not bad.any(), (s, q[s][bad], Qo[bad])


def test_static_entry_point_specialised_kernels_and_one_loop():
    print("static scratch: specialised kernels; one-loop sector", flush=True)
    prob = W.two_loop_integral(seed=6, n_sectors=6, n_scale=0.01, m=8)
    ref, st = _pair(prob)
    ref.specialize()
    st.specialize()
    _compare(ref, st)
    _compare(*_pair(W.one_loop_sector(seed=0, n=4099, m=8)))


def test_static_entry_point_rejects_oversized_call():
    import paper_2305_19768_amd as qmc
    from paper_2305_19768_amd import _abi
    print("static scratch: oversized launch rejected on the host", flush=True)
    prob = W.two_loop_integral(seed=7, n_sectors=4, m=64)
    st = qmc.Plan(prob, bind_workspace=False, shift_tile=16)
    # 32768 target workgroups x 16 shifts x 3 orders x 16 B is over the 16 MiB array
    st.set_launch_shape(block=256, shift_tile=16, shifts_per_pass=2, target_blocks=32768)
    with pytest.raises(qmc.QmcError, match="static scratch"):
        st.integrate_static()
    assert _abi.lib().qmc_integrate_static(None, None, None, None, None, None, None) == -1
    # a call that fits still runs after the rejection
    st.set_launch_shape(block=256, shift_tile=16, shifts_per_pass=2, target_blocks=1024)
    ref = qmc.Plan(prob, shift_tile=16)
    ref.set_launch_shape(block=256, shift_tile=16, shifts_per_pass=2, target_blocks=1024)
    _compare(ref, st)
