"""dg_step on a run that turns non-physical: the step in which a kernel
meets a non-physical state is the last one, and the call reports it with the
time and step count after that step (the batched path stops such an
instance the same way)."""
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_step_stops_after_the_step_that_meets_a_nonphysical_state():
    from paper_1904_11147_amd import dg
    from paper_1904_11147_amd import workloads as W
    # the Q3 instance of the benchmark batch (98^2, seed 10195) that loses
    # positivity within 200 steps without the positivity scaling
    wl = [w for w in W.riemann2d_batch() if w.seed == 10195][0]
    p = dg.problem_from_workload(wl)
    s0 = dg.initial_state(p, wl, limit=True)
    assert p.status() == dg.DG_OK
    a = s0.clone()
    t, k = p.step(a, 0.0, wl.t_end, max_steps=200, allow_nonphysical=True)
    assert p.status() == dg.DG_ERR_NONPHYSICAL and p.status() == dg.DG_OK  # sticky until read once
    assert 1 < k < 200 and 0.0 < t < wl.t_end, (k, t)
    b = s0.clone()
    t1, k1 = p.step(b, 0.0, wl.t_end, max_steps=k - 1)  # raises if a step before k were non-physical
    assert k1 == k - 1 and t1 < t
    with pytest.raises(dg.DGError) as e:
        p.step(b, t1, wl.t_end, max_steps=50)
    assert e.value.code == dg.DG_ERR_NONPHYSICAL
    p.status()
    c = s0.clone()
    t2, k2 = p.step(c, 0.0, wl.t_end, max_steps=k - 1)
    t3, k3 = p.step(c, t2, wl.t_end, max_steps=50, allow_nonphysical=True)
    assert k3 == 1 and t3 == t, (k3, t3, t)
    assert torch.equal(a, c)
    p.close()
