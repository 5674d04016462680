"""Batched stepping and the strip-height autotuner (GPU).

A lattice advanced inside a batch of other lattices (different sizes,
fluids, geometries), with plain launches or HIP-graph replays, must give the
bitwise same populations as the lattice advanced alone; so must a lattice
whose strip height was retuned mid-run."""
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


def problems():
    return [W.reduction_case(), W.random_fields(100, 37, geometry="channel", U=0.01),
            W.random_fields(130, 70, geometry="cylinder", rho=(3.0, 2.0, 1.0)),
            W.binary_drops(seed=3, nx=128, ny=64, R=16),
            W.random_fields(70, 50, geometry="box")]


@pytest.mark.parametrize("precision,graph", [("fp64", 0), ("fp64", 16), ("fp32", 8),
                                             ("fp16dev", 0)])
def test_batch_bitwise_equals_solo(tlb, precision, graph):
    probs = problems()
    steps = 101
    solo = []
    for p in probs:
        s = tlb.from_problem(p, precision)
        s.set_check_interval(0)
        s.step(steps)
        solo.append(s.read_populations())
    members = [tlb.from_problem(p, precision) for p in probs]
    b = tlb.Batch(8)
    b.set(members)
    if graph:
        b.use_graph(graph)
    b.step(40)
    b.step(steps - 40)
    b.sync()
    for s, ref in zip(members, solo):
        assert s.step_count == steps
        assert np.array_equal(s.read_populations(), ref)


def test_batch_rejects_member_stepped_alone(tlb):
    probs = problems()[:2]
    members = [tlb.from_problem(p) for p in probs]
    b = tlb.Batch(4)
    b.set(members)
    b.step(3)
    b.sync()
    members[0].step(1)
    with pytest.raises(tlb.TlbError) as e:
        b.step(1)
    assert e.value.status == tlb.TLB_ESTATE
    b.set(members)          # re-registering picks up the new state
    b.step(2)
    b.sync()


def test_batch_rejects_mixed_precision(tlb):
    probs = problems()[:2]
    members = [tlb.from_problem(probs[0], "fp64"), tlb.from_problem(probs[1], "fp32")]
    b = tlb.Batch(4)
    with pytest.raises(tlb.TlbError) as e:
        b.set(members)
    assert e.value.status == tlb.TLB_EINVAL


def test_autotune_keeps_the_trajectory(tlb):
    p = W.random_fields(130, 70, geometry="cylinder")
    a = tlb.from_problem(p)
    a.set_check_interval(0)
    best = a.autotune_rows(5)
    n = a.step_count
    assert best % 4 == 0 and n > 0
    b = tlb.from_problem(p)
    b.set_check_interval(0)
    b.step(n)
    assert np.array_equal(a.read_populations(), b.read_populations())


def test_batch_autotune_keeps_the_trajectory(tlb):
    """The batch autotuner (one strip height per size class, chosen by timing
    the batched launch) advances every member but leaves its trajectory
    bitwise that of the member stepped alone for the same number of steps,
    and gives each class a legal strip height."""
    probs = problems()
    members = [tlb.from_problem(p, "fp32") for p in probs]
    for s in members:
        s.set_check_interval(0)
    b = tlb.Batch(8)
    b.set(members)
    best = b.autotune_rows(3)
    b.step(7)
    b.sync()
    assert best % 4 == 0 and 16 <= best <= 128
    for p, s in zip(probs, members):
        n = s.step_count
        assert n > 7
        ref = tlb.from_problem(p, "fp32")
        ref.set_check_interval(0)
        ref.step(n)
        assert np.array_equal(s.read_populations(), ref.read_populations()), p["name"]


def test_batch_with_optional_features_equals_oracle(tlb):
    """One FP64 batch of a plain lattice with scattered obstacles, a channel with
    a velocity boundary (Eqs. 51-53) and a lattice with lambda > 0 (Eqs. 5-6):
    the launch runs the kernel variant with both optional parts for every
    member, and each member must still equal the FP64 oracle within 1e-12 on
    every field and population."""
    import oracle
    plain = W.random_obstacles(96, 70, seed=8, n_obstacles=25)
    vel = W.random_fields(100, 37, geometry="channel", U=0.01, rho=(3.0, 2.0, 1.0), seed=9)
    vel = dict(vel, mats=[vel["mats"][0], W.velocity_boundary((0.02, 0.0))], name=vel["name"] + "_v")
    lam = W.random_fields(64, 40, geometry="cylinder", rho=(3.0, 2.0, 1.0), seed=10)
    lam["fluid"] = dict(lam["fluid"], **{"lambda": 2e-2})
    probs = [plain, vel, lam, W.reduction_case()]
    steps = 201
    members = [tlb.from_problem(p, "fp64") for p in probs]
    b = tlb.Batch(8)
    b.set(members)
    b.step(steps)
    b.sync()
    for p, s in zip(probs, members):
        o = oracle.Oracle(p)
        o.init(p["c1"], p["c2"], p["ux"], p["uy"])
        o.step(steps)
        fg, fo = s.read_fields(), o.fields()
        e = {k: float(np.abs(fg[k] - fo[k]).max()) for k in fo}
        print("batch member %s: %s" % (p["name"], {k: "%.1e" % v for k, v in e.items()}), flush=True)
        assert max(e.values()) <= 1e-12, (p["name"], e)
        po = o.populations()
        po[:, o.material != 0] = 0.0
        assert np.abs(s.read_populations() - po).max() <= 1e-12, p["name"]
