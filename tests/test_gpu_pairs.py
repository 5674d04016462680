"""The two-step kernel (tlb_set_pair_rows): one launch advances the lattice by
two time steps, the first level keeping its post-collision populations in
LDS.  Every node of both levels goes through the same arithmetic as a step of
the one-step kernel, so the state after any number of steps must be bitwise
identical with pairs on and off: populations, fields and history (the mass
read from it), on walls moving along both axes, scattered obstacles touching
strip boundaries and the periodic seams, density contrast with gravity,
the bulk energy with lambda > 0, velocity boundary nodes, ragged last strips
and several strip heights, odd step counts (a pair
sequence ending in a single step) and health checks that split pairs.  Also
against the FP64 oracle within the FP32 bar, at the benchmark's 1024 x 2048
lattice, and the argument checks of the entry point.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1710_09534_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_09534_amd import tlb as t
    return t


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _with_lambda(p, lam):
    p["fluid"] = dict(p["fluid"], **{"lambda": lam})
    return p


def _cases():
    return {
        "obstacles_128x96": lambda: W.random_obstacles(128, 96, seed=3, n_obstacles=30),
        "channel_192x70_rho_g": lambda: W.random_fields(192, 70, seed=9, geometry="channel", U=0.01,
                                                        rho=(10.0, 5.0, 1.0), gravity=(0.0, -1e-6)),
        "box_64x40": lambda: W.random_fields(64, 40, seed=4, geometry="box", U=0.01),
        # the optional parts: bulk energy with lambda > 0 (Eqs. 5-6), and
        # velocity boundary nodes (Eqs. 51-53) in the top row
        "lambda_128x96": lambda: _with_lambda(
            W.random_fields(128, 96, seed=5, geometry="channel", U=0.01), 0.05),
        "velocity_448x72": lambda: W.nee_shear(nx=448, ny=72, R_core=10.0, R_shell=24.0, offset=3.0),
    }


def _state(g):
    return g.read_populations(), g.read_fields(), g.mass()


def _assert_same(a, b, what):
    pa, fa, ma = a
    pb, fb, mb = b
    assert np.array_equal(pa, pb), "%s: populations differ, max %.3e" % (
        what, float(np.abs(pa - pb).max()))
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), "%s: field %s differs" % (what, k)
    assert np.array_equal(ma, mb), what


@pytest.mark.parametrize("name", sorted(_cases()))
@pytest.mark.parametrize("rows", [8, 12, 32])
def test_pairs_bitwise_equal_single_steps(tlb, name, rows):
    p = _cases()[name]()
    steps = 9
    _say("case %s fp32 pairs rows=%d %d steps" % (name, rows, steps))
    ref = tlb.from_problem(p, "fp32")
    ref.set_pair_rows(0)
    ref.step(steps)
    a = _state(ref)
    g = tlb.from_problem(p, "fp32")
    g.set_pair_rows(rows)
    g.step(steps)
    assert g.step_count == steps
    _assert_same(_state(g), a, "%s rows=%d" % (name, rows))


def _ragged_cases():
    return {
        "obstacles_100x96": lambda: W.random_obstacles(100, 96, seed=31, n_obstacles=20),
        "channel_130x70_rho_g": lambda: W.random_fields(130, 70, seed=32, geometry="channel", U=0.01,
                                                        rho=(10.0, 5.0, 1.0), gravity=(0.0, -1e-6)),
        "box_40x24": lambda: W.random_fields(40, 24, seed=33, geometry="box", U=0.01),
        "periodic_127x33": lambda: W.random_fields(127, 33, seed=34, geometry="periodic"),
        "periodic_5x17": lambda: W.random_fields(5, 17, seed=35, geometry="periodic"),
        "lambda_150x40": lambda: _with_lambda(
            W.random_fields(150, 40, seed=36, geometry="channel", U=0.01), 0.05),
        "velocity_430x72": lambda: W.nee_shear(nx=430, ny=72, R_core=10.0, R_shell=24.0, offset=3.0),
    }


@pytest.mark.parametrize("name", sorted(_ragged_cases()))
@pytest.mark.parametrize("rows", [8, 32])
def test_pairs_ragged_widths(tlb, name, rows):
    """Widths that are not a multiple of 64 (and one narrower than a strip):
    in the last strip the lanes past nx step the wrapped columns that are the
    strip's right frame, and store nothing; 7 steps (three two-step launches
    and one single) are bitwise those of 7 single steps."""
    p = _ragged_cases()[name]()
    _say("case %s pairs rows=%d, 7 steps" % (p["name"], rows))
    ref = tlb.from_problem(p, "fp32")
    ref.set_pair_rows(0)
    ref.step(7)
    g = tlb.from_problem(p, "fp32")
    g.set_pair_rows(rows)
    g.step(7)
    _assert_same(_state(g), _state(ref), "%s rows=%d" % (name, rows))


def test_pairs_ragged_full_size(tlb):
    """A 1000 x 2048 cylinder-impact lattice (16 strip columns, the last 40
    columns wide) at its default two-step strips: 20 steps bitwise those of
    20 single steps."""
    p = W.cylinder_impact(nx=1000, ny=2048)
    _say("case %s default pairs, 20 steps" % p["name"])
    ref = tlb.from_problem(p, "fp32")
    ref.set_pair_rows(0)
    ref.step(20)
    g = tlb.from_problem(p, "fp32")
    g.step(20)
    _assert_same(_state(g), _state(ref), "cylinder 1000x2048")


@pytest.mark.parametrize("geometry,ny", [("channel", 12), ("periodic", 16), ("channel", 3),
                                         ("periodic", 3), ("periodic", 5), ("channel", 6)])
def test_pairs_short_lattices(tlb, geometry, ny):
    """Lattices shorter than a strip's frame (a 8-row strip's first level
    spans 16 rows): the first level wraps the periodic seam onto rows it also
    computes elsewhere in the ring, several times over for lattices shorter
    than the strip itself; still bitwise equal to single steps."""
    p = W.random_fields(128, ny, seed=11, geometry=geometry, U=0.01)
    _say("case %s pairs rows=8, 7 steps" % p["name"])
    ref = tlb.from_problem(p, "fp32")
    ref.set_pair_rows(0)
    ref.step(7)
    g = tlb.from_problem(p, "fp32")
    g.set_pair_rows(8)
    g.step(7)
    _assert_same(_state(g), _state(ref), "%s ny=%d" % (geometry, ny))


def test_pairs_split_by_health_checks(tlb):
    """With a check every 3 steps, 10 steps run as pair, single (check),
    pair, single (check), ...: still the same state, and stepping on from a
    checkpoint taken mid-way continues identically."""
    p = W.random_obstacles(128, 96, seed=5, n_obstacles=25)
    _say("case %s pairs with check interval 3" % p["name"])
    ref = tlb.from_problem(p, "fp32")
    ref.set_pair_rows(0)
    ref.set_check_interval(3)
    ref.step(10)
    g = tlb.from_problem(p, "fp32")
    g.set_check_interval(3)
    g.set_pair_rows(16)
    g.step(10)
    _assert_same(_state(g), _state(ref), "check interval 3")
    blob = g.checkpoint_save()
    h = tlb.from_problem(p, "fp32", init=False)
    h.checkpoint_load(blob)
    h.set_pair_rows(16)
    h.step(5)
    ref.step(5)
    _assert_same(_state(h), _state(ref), "after checkpoint")


def test_batch_after_pairs(tlb):
    """A context left on its second history set by an odd number of two-step
    launches joins a batch (one step per launch, history updated in place in
    that set), and a second batch member is stepped outside the batch in
    between, which the batch must refuse: the members end bitwise equal to
    contexts stepped one step at a time throughout."""
    p = W.random_obstacles(128, 96, seed=7, n_obstacles=20)
    q = W.random_fields(192, 64, seed=2, geometry="channel", U=0.01)
    refs = []
    for prob in (p, q):
        r = tlb.from_problem(prob, "fp32")
        r.set_pair_rows(0)
        r.step(9)
        refs.append(_state(r))
    a = tlb.from_problem(p, "fp32")
    a.set_pair_rows(16)
    a.step(2)                    # one two-step launch: current history is set 1
    b = tlb.from_problem(q, "fp32")
    b.set_pair_rows(0)
    b.step(2)
    batch = tlb.Batch(4)
    batch.set([a, b])
    batch.step(5)
    batch.sync()
    a.step(2)                    # outside the batch: another two-step launch
    with pytest.raises(tlb.TlbError):
        batch.step(1)            # a member moved on without the batch
    b.step(2)
    _assert_same(_state(a), refs[0], "pairs, batch, pairs")
    _assert_same(_state(b), refs[1], "batch member")


def _solo_refs(tlb, probs, precision, steps):
    refs = []
    for prob in probs:
        r = tlb.from_problem(prob, precision)
        r.set_pair_rows(0)
        r.step(steps)
        refs.append(_state(r))
    return refs


@pytest.mark.parametrize("rows", [16, 64])
def test_batch_pairs_bitwise(tlb, rows):
    """A batch of lattices of several sizes, geometries and optional parts,
    two steps per launch over strips of `rows` rows of every member (taller
    than some lattices): 9 batched steps (four two-step launches and one
    single) equal the same batch stepped one step per launch.  (A batch that
    mixes optional parts runs every member through the kernel instance with
    all of them, so a plain member's reference is the batch, not the member
    alone; the plain-only batches below compare with members alone.)"""
    probs = [_cases()[k]() for k in sorted(_cases())] + [W.reduction_case(nx=64, ny=64)]
    states = []
    for pr in (0, rows):
        members = [tlb.from_problem(p, "fp32") for p in probs]
        batch = tlb.Batch(8)
        batch.set(members)
        batch.set_pair_rows(pr)
        batch.step(9)
        batch.sync()
        states.append([_state(m) for m in members])
    for p, a, b in zip(probs, states[1], states[0]):
        _assert_same(a, b, "batch pairs rows=%d %s" % (rows, p["name"]))


def test_batch_pairs_plain_members_equal_alone(tlb):
    """Plain members (no optional part in the batch): two steps per launch in
    the batch equal each member alone one step per launch."""
    probs = [W.random_obstacles(128, 96, seed=3, n_obstacles=30),
             W.random_fields(192, 70, seed=9, geometry="channel", U=0.01, rho=(10.0, 5.0, 1.0),
                             gravity=(0.0, -1e-6)),
             W.random_fields(64, 40, seed=4, geometry="box"), W.reduction_case(nx=64, ny=64)]
    refs = _solo_refs(tlb, probs, "fp32", 9)
    members = [tlb.from_problem(p, "fp32") for p in probs]
    batch = tlb.Batch(4)
    batch.set(members)
    batch.set_pair_rows(32)
    batch.step(9)
    batch.sync()
    for p, m, r in zip(probs, members, refs):
        _assert_same(_state(m), r, "plain batch pairs %s" % p["name"])


def test_batch_pairs_default_rows_short_members(tlb):
    """The batch default (each member's strip: its height rounded up to 4,
    at least 8 and at most 128 rows) with members 3 and 5 rows high beside
    taller ones: 9 batched steps equal each member alone one step per
    launch."""
    probs = [W.random_fields(128, 3, seed=21, geometry="periodic"),
             W.random_fields(64, 5, seed=22, geometry="periodic"),
             W.random_fields(128, 6, seed=23, geometry="channel", U=0.01),
             W.random_obstacles(128, 96, seed=24, n_obstacles=20), W.reduction_case(nx=64, ny=64)]
    refs = _solo_refs(tlb, probs, "fp32", 9)
    members = [tlb.from_problem(p, "fp32") for p in probs]
    batch = tlb.Batch(5)
    batch.set(members)
    batch.step(9)
    batch.sync()
    for p, m, r in zip(probs, members, refs):
        _assert_same(_state(m), r, "default-row batch pairs %s" % p["name"])


def test_batch_autotune_pair_rows_keeps_trajectory(tlb):
    """The two-step batch tuner times candidate strip heights per size class
    on the batched launch: the members advance by the timed steps, stay
    bitwise those of lone single steps, keep the tuned heights through a
    re-registration and lose them at set_pair_rows; an FP64 batch (one step
    per launch) is refused."""
    probs = [W.random_obstacles(128, 96, seed=41, n_obstacles=20), W.reduction_case(nx=64, ny=64),
             W.random_fields(100, 40, seed=42, geometry="box")]
    members = [tlb.from_problem(p, "fp32") for p in probs]
    batch = tlb.Batch(3)
    batch.set(members)
    best = batch.autotune_pair_rows(3)        # 4 steps per candidate
    assert best in (8, 16, 32, 64, 128)
    n = members[0].step_count
    assert n > 0 and n % 4 == 0 and all(m.step_count == n for m in members)
    batch.set(members)
    batch.step(5)
    batch.set_pair_rows(-1)
    batch.step(3)
    batch.sync()
    refs = _solo_refs(tlb, probs, "fp32", n + 8)
    for p, m, r in zip(probs, members, refs):
        _assert_same(_state(m), r, "tuned batch pairs %s" % p["name"])
    f64 = [tlb.from_problem(p, "fp64") for p in probs[1:]]
    b64 = tlb.Batch(2)
    b64.set(f64)
    with pytest.raises(tlb.TlbError):
        b64.autotune_pair_rows(2)


def test_batch_pairs_graph(tlb):
    """Graph replay of two-step launches (a multiple of 4 steps) between
    plain launches: 22 batched steps equal 22 single steps; a graph of 6
    steps is refused while pairs are on."""
    probs = [W.random_obstacles(128, 96, seed=12, n_obstacles=20), W.reduction_case(nx=64, ny=64)]
    refs = _solo_refs(tlb, probs, "fp32", 22)
    members = [tlb.from_problem(p, "fp32") for p in probs]
    batch = tlb.Batch(2)
    batch.set(members)
    batch.set_pair_rows(32)
    with pytest.raises(tlb.TlbError):
        batch.use_graph(6)
    batch.use_graph(8)
    batch.step(1)      # off parity: plain launches until the next multiple of the graph
    batch.step(21)
    batch.sync()
    for p, m, r in zip(probs, members, refs):
        _assert_same(_state(m), r, "batch graph pairs %s" % p["name"])


def test_batch_pairs_not_applicable(tlb):
    """FP64 members keep one step per launch when pairs are asked for, with
    the same results; an FP32 batch with a 100-column member takes pairs and
    equals its members alone."""
    probs = [W.random_fields(64, 40, seed=4, geometry="box"), W.reduction_case(nx=64, ny=64)]
    refs = _solo_refs(tlb, probs, "fp64", 5)
    members = [tlb.from_problem(p, "fp64") for p in probs]
    batch = tlb.Batch(2)
    batch.set(members)
    batch.set_pair_rows(16)
    batch.step(5)
    batch.sync()
    for p, m, r in zip(probs, members, refs):
        _assert_same(_state(m), r, "fp64 batch %s" % p["name"])
    q = [W.random_fields(100, 40, seed=4, geometry="box"), W.reduction_case(nx=64, ny=64)]
    refs = _solo_refs(tlb, q, "fp32", 5)
    members = [tlb.from_problem(p, "fp32") for p in q]
    batch = tlb.Batch(2)
    batch.set_pair_rows(16)
    batch.set(members)
    batch.step(5)
    batch.sync()
    for p, m, r in zip(q, members, refs):
        _assert_same(_state(m), r, "mixed-width fp32 batch %s" % p["name"])


def test_pairs_time_steps_equal_steps(tlb):
    """tlb_time_steps advances the state with the same launches as tlb_step."""
    p = W.random_obstacles(128, 96, seed=6, n_obstacles=20)
    ref = tlb.from_problem(p, "fp32")
    ref.set_pair_rows(0)
    ref.step(8)
    g = tlb.from_problem(p, "fp32")
    g.set_pair_rows(24)
    ms = g.time_steps(8)
    assert ms > 0.0
    _assert_same(_state(g), _state(ref), "time_steps")


def test_pairs_against_oracle(tlb):
    """300 steps of moving obstacles in pairs against the FP64 oracle: the
    FP32 bar of the other parity tests (order parameters within 1e-4)."""
    p = W.random_obstacles(192, 128, seed=8, n_obstacles=40)
    o = oracle.Oracle(p)
    o.init(p["c1"], p["c2"], p["ux"], p["uy"])
    o.step(300)
    fo = o.fields()
    g = tlb.from_problem(p, "fp32")
    g.set_pair_rows(32)
    g.step(300)
    fg = g.read_fields()
    e = {k: float(np.abs(fg[k] - fo[k]).max()) for k in fo}
    _say("pairs fp32 vs oracle: %s" % {k: "%.1e" % v for k, v in e.items()})
    assert e["c1"] <= 1e-4 and e["c2"] <= 1e-4 and e["c3"] <= 1e-4, e


def test_pairs_full_size_cylinder(tlb):
    """The benchmark lattice (1024 x 2048 cylinder impact, FP32) with the
    default pair strip height (the default mode): 2001 steps (1000 two-step
    launches, health checks every 100 steps, a last single step) equal 2001
    single steps bitwise, and conserve each component's mass to FP32
    round-off (relative 1e-5 over the 2001 steps)."""
    p = W.cylinder_impact(nx=1024, ny=2048)
    _say("case %s pairs default rows, 2001 steps" % p["name"])
    ref = tlb.from_problem(p, "fp32")
    ref.set_pair_rows(0)
    m0 = ref.mass()
    ref.step(2001)
    a = _state(ref)
    del ref
    g = tlb.from_problem(p, "fp32")
    g.step(2001)
    st = _state(g)
    _assert_same(st, a, "cylinder 1024x2048")
    rel = np.abs(st[2] - m0) / np.abs(m0)
    _say("mass drift after 2001 steps: %s" % rel)
    assert rel.max() <= 1e-5, rel


def test_pair_rows_arguments(tlb):
    p = W.random_fields(64, 40, seed=4, geometry="box")
    g64 = tlb.from_problem(p, "fp64")
    with pytest.raises(tlb.TlbError):
        g64.set_pair_rows(16)
    g64.set_pair_rows(-1)   # the default; not applicable: one step per launch
    g64.set_pair_rows(0)
    g64.step(2)
    g32 = tlb.from_problem(p, "fp32")
    for bad in (4, 10, 8192, -2):
        with pytest.raises(tlb.TlbError):
            g32.set_pair_rows(bad)
    q = W.random_fields(100, 40, seed=4, geometry="box")
    tlb.from_problem(q, "fp32").set_pair_rows(16)      # any width
    h = tlb.from_problem(W.random_fields(64, 40, seed=4, geometry="box"), "fp16dev")
    with pytest.raises(tlb.TlbError):
        h.set_pair_rows(16)
    # optional step parts are served by the two-step kernel too
    tlb.from_problem(W.nee_shear(nx=448, ny=72, R_core=10.0, R_shell=24.0), "fp32").set_pair_rows(16)
