"""Continuous-batching server (GPU): results identical alone and in a mix,
admission under a small HBM arena, cancellation, failure isolation."""
import numpy as np
import pytest

from paper_1710_09534_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_09534_amd import tlb as t
    return t


def mix(n=8, seed=11):
    rng = W.Rng(seed)
    sizes = [64, 96, 128, 64, 160, 64, 128, 96, 64, 128]
    out = []
    for i in range(n):
        p = W.serving_request(W.Rng(rng.next_u64()), sizes[i % len(sizes)], i % 3, (150, 600))
        out.append(p)
    return out


def solo(tlb, p, precision):
    s = tlb.from_problem(p, precision)
    s.set_check_interval(0)
    s.step(p["steps"])
    return s.read_fields()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
def test_results_identical_alone_and_in_mix(tlb, precision):
    probs = mix()
    # an arena that holds only a few lattices at a time forces queueing and
    # admission as earlier requests finish
    ws = max(tlb.tlb_workspace_bytes(p["nx"], p["ny"], tlb.PRECISIONS[precision]) for p in probs)
    srv = tlb.Server(3 * ws + (1 << 20), max_slots=3, precision=precision, quantum=100)
    ids = [srv.submit(p, p["steps"]) for p in probs]
    for i in ids:
        srv.wait(i, 120.0)
    st = srv.stats()
    assert st["completed"] == len(probs) and st["failed"] == 0
    for p, i in zip(probs, ids):
        f, lat = srv.result(i, p["nx"], p["ny"])
        assert lat > 0
        ref = solo(tlb, p, precision)
        for k in ref:
            assert np.array_equal(f[k], ref[k]), (p["name"], k)
    srv.close()


def test_oversized_request_rejected(tlb):
    p = mix(1)[0]
    srv = tlb.Server(1 << 20, max_slots=2, precision="fp32")
    with pytest.raises(tlb.TlbError) as e:
        srv.submit(p, 10)
    assert e.value.status == tlb.TLB_ENOMEM
    srv.close()


def test_cancel_and_failure_isolation(tlb):
    probs = mix(3)
    bad = dict(probs[1])
    bad["fluid"] = dict(bad["fluid"], gravity=[0.0, -50.0])  # diverges
    inadmissible = dict(probs[1])
    inadmissible["fluid"] = dict(inadmissible["fluid"], tau1=0.4)  # tau_i <= 1/2
    srv = tlb.Server(1 << 30, max_slots=4, precision="fp64", quantum=50)
    ok_id = srv.submit(probs[0], 300)
    bad_id = srv.submit(bad, 400)
    rej_id = srv.submit(inadmissible, 100)
    long_id = srv.submit(probs[2], 10 ** 7)
    srv.wait(ok_id, 120.0)
    srv.wait(bad_id, 120.0)
    srv.wait(rej_id, 120.0)
    assert srv.poll(ok_id) == tlb.TLB_REQ_DONE
    assert srv.poll(bad_id) == tlb.TLB_REQ_FAILED
    assert srv.poll(rej_id) == tlb.TLB_REQ_FAILED
    # each failed request reports what failed it
    with pytest.raises(tlb.TlbError) as e:
        srv.result(bad_id, bad["nx"], bad["ny"])
    assert e.value.status == tlb.TLB_EDIVERGED
    with pytest.raises(tlb.TlbError) as e:
        srv.result(rej_id, bad["nx"], bad["ny"])
    assert e.value.status == tlb.TLB_EPARAM and "tau" in str(e.value)
    srv.cancel(long_id)
    srv.wait(long_id, 120.0)
    assert srv.poll(long_id) == tlb.TLB_REQ_CANCELLED
    with pytest.raises(ValueError):   # a host buffer sized for another lattice is refused
        srv.result(ok_id, probs[0]["nx"] + 1, probs[0]["ny"])
    f, _ = srv.result(ok_id, probs[0]["nx"], probs[0]["ny"])
    p0 = dict(probs[0], steps=300)
    ref = solo(tlb, p0, "fp64")
    assert np.array_equal(f["c1"], ref["c1"])
    srv.close()


def test_diverged_request_fails_early(tlb):
    """A request driven unstable by an absurd body force fails at the first
    periodic health check after it diverges, long before its step budget,
    while a well-posed request in the same mix finishes with its solo result."""
    import time
    probs = mix(2)
    bad = dict(probs[1])
    bad["fluid"] = dict(bad["fluid"], gravity=[0.0, -50.0])
    srv = tlb.Server(1 << 30, max_slots=4, precision="fp32", quantum=50)
    srv.set_check_steps(100)
    t0 = time.perf_counter()
    bad_id = srv.submit(bad, 10 ** 8)          # would take hours if it ran to the end
    ok_id = srv.submit(probs[0], 300)
    srv.wait(bad_id, 120.0)
    assert srv.poll(bad_id) == tlb.TLB_REQ_FAILED
    assert time.perf_counter() - t0 < 60.0
    with pytest.raises(tlb.TlbError) as e:
        srv.result(bad_id, bad["nx"], bad["ny"])
    assert e.value.status == tlb.TLB_EDIVERGED
    srv.wait(ok_id, 120.0)
    assert srv.poll(ok_id) == tlb.TLB_REQ_DONE
    f, _ = srv.result(ok_id, probs[0]["nx"], probs[0]["ny"])
    ref = solo(tlb, dict(probs[0], steps=300), "fp32")
    assert np.array_equal(f["c1"], ref["c1"])
    srv.close()
