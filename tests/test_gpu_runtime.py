"""GPU checks of the runtime forms of the step: hipGraph replay, the batched
launch over uneven cases, and the autotuner (all must reproduce plain
single-case launches bit for bit)."""
import numpy as np
import pytest

from paper_2207_09431_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Solver():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2207_09431_amd.pflbm import Solver as S
    return S


def fields(s, k=0):
    m = s.macroscopic(k)
    s.synchronize()
    return {n: v.cpu().numpy() for n, v in m.items()}


def same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("u", "p", "phi", "rho"))


def test_graph_replay_matches_plain_launches(Solver):
    case = inputs.rising_bubble_small()
    ref = Solver(case["params"])
    ref.init_fields(0, case["C"], case["u"], case["p"])
    g = Solver(case["params"])
    g.init_fields(0, case["C"], case["u"], case["p"])
    g.set_graph(6)
    # an odd first call leaves the state on the other parity before the graph runs
    for n in (3, 13, 6, 20):
        ref.step(n)
        g.step(n)
        a, b = fields(ref), fields(g)
        print("after", n, "steps: bitwise equal", same(a, b), flush=True)
        assert same(a, b)


def test_batched_cases_match_single_runs(Solver):
    cases = [inputs.rising_bubble_small(), inputs.static_bubble(nx=70, ny=45, radius=12.0),
             inputs.powerlaw_bubble(n=0.7, nx=100, ny=200, d=50.0)]
    batch = Solver([c["params"] for c in cases])
    for k, c in enumerate(cases):
        batch.init_fields(k, c["C"], c["u"], c["p"])
    batch.step(40)
    for k, c in enumerate(cases):
        one = Solver(c["params"])
        one.init_fields(0, c["C"], c["u"], c["p"])
        one.step(40)
        assert same(fields(batch, k), fields(one)), c["name"]
        a = batch.bubble_centroid_velocity(k, 0)
        b = one.bubble_centroid_velocity(0, 0)
        assert np.array_equal(a, b)


def test_autotune_leaves_state_and_results_unchanged(Solver, tmp_path):
    case = inputs.rising_bubble_small()
    ref = Solver(case["params"])
    ref.init_fields(0, case["C"], case["u"], case["p"])
    ref.step(7)
    t = Solver(case["params"])
    t.init_fields(0, case["C"], case["u"], case["p"])
    t.step(7)
    name = t.autotune(steps=3, cache=str(tmp_path / "tune.json"))
    print("chosen", name, t.tuning, flush=True)
    assert same(fields(ref), fields(t))
    ref.step(11)
    t.step(11)
    assert same(fields(ref), fields(t))
    # the cache answers without timing again
    again = Solver(case["params"])
    again.init_fields(0, case["C"], case["u"], case["p"])
    assert again.autotune(steps=3, cache=str(tmp_path / "tune.json")) == name


def test_checkpoints_of_two_runs_are_bitwise_equal(Solver):
    """get_state copies whole planes, row padding included; the workspace
    starts zeroed, so two runs from the same inputs give identical bytes."""
    case = inputs.static_bubble(nx=70, ny=45, radius=12.0)
    states = []
    for _ in range(2):
        s = Solver(dict(case["params"], store_h=1))
        s.init_fields(0, case["C"], inputs.velocity_noise(70, 45, 3, 1e-3), None)
        s.step(9)
        states.append(s.get_state().cpu().numpy())
        s.close()
    assert np.array_equal(states[0], states[1])


def _status(call):
    from paper_2207_09431_amd.pflbm import PflbmError
    try:
        call()
    except PflbmError as e:
        return e.status
    return 0


def test_nonfinite_flag_is_sticky(Solver):
    """A NaN planted in a copy of the state (level s of one node) through
    set_state: the next synchronising calls return NONFINITE (-4) and keep
    doing so; stepping stays possible (asynchronous); set_state with a finite
    state or init_fields clears the flag.  A NaN only in tau is found by the
    state scan."""
    import torch
    case = inputs.rising_bubble_small()
    s = Solver(case["params"])
    s.init_fields(0, case["C"], case["u"], case["p"])
    s.step(3)
    good = s.get_state()
    assert _status(s.check_state) == 0
    bad = good.clone()
    bad.view(torch.float64)[200] = float("nan")      # the level plane comes first
    s.set_state(bad)
    assert not s.case_nonfinite(0)
    assert _status(lambda: s.bubble_centroid_velocity(0, 0)) == -4
    assert s.case_nonfinite(0)
    assert _status(s.check_state) == -4
    assert _status(lambda: s.bubble_centroid_velocity(0, 2)) == -4
    s.step(2)
    assert _status(s.check_state) == -4
    s.set_state(good)
    assert _status(s.check_state) == 0 and not s.case_nonfinite(0)
    assert _status(lambda: s.bubble_centroid_velocity(0, 0)) == 0
    # macroscopic (asynchronous) marks the device flag; the next synchronising call reports it
    s.set_state(bad)
    s.macroscopic(0)
    s.synchronize()
    assert not s.case_nonfinite(0)
    assert _status(lambda: s.bubble_centroid_velocity(0, 0)) == -4
    s.init_fields(0, case["C"], case["u"], case["p"])
    assert _status(s.check_state) == 0
    # a NaN confined to tau (the last plane of the state)
    taubad = good.clone()
    tv = taubad.view(torch.float32)
    tv[tv.numel() - 1000] = float("nan")
    s.set_state(taubad)
    assert _status(s.check_state) == -4


def test_nonfinite_flag_is_per_case(Solver):
    """In a batch, a non-finite case does not flag the others, which can be
    advanced and reduced; init_fields of the bad case clears it."""
    import torch
    cases = [inputs.rising_bubble_small(), inputs.static_bubble(nx=70, ny=45, radius=12.0)]
    b = Solver([c["params"] for c in cases])
    for k, c in enumerate(cases):
        b.init_fields(k, c["C"], c["u"], c["p"])
    good = b.get_state()
    bad = good.clone()
    bad.view(torch.float64)[100] = float("inf")      # case 0 comes first in the state
    b.set_state(bad)
    assert _status(b.check_state) == -4
    assert b.case_nonfinite(0) and not b.case_nonfinite(1)
    b.step(4)
    assert _status(lambda: b.bubble_centroid_velocity(1, 0)) == 0
    assert _status(lambda: b.bubble_centroid_velocity(0, 0)) == -4
    b.init_fields(0, cases[0]["C"], cases[0]["u"], cases[0]["p"])
    assert _status(b.check_state) == 0


def test_centroid_arguments(Solver):
    """Component 1 (C_2) is not carried with one phase field (INVALID_ARG);
    a component with zero mass has no centroid (NONFINITE, not sticky)."""
    import numpy as np
    case = inputs.rising_bubble_small()
    s = Solver(case["params"])
    s.init_fields(0, case["C"], case["u"], case["p"])
    assert _status(lambda: s.bubble_centroid_velocity(0, 1)) == -1
    s.init_fields(0, np.zeros_like(case["C"]))
    assert _status(lambda: s.bubble_centroid_velocity(0, 0)) == -4
    assert not s.case_nonfinite(0)
    assert _status(s.check_state) == 0
    assert s.bubble_centroid_velocity(0, 2)[0] == 64 * 128


def test_init_fields_rejects_wrong_shapes(Solver):
    """The binding checks the shapes of the host fields against the case
    before the ABI reads nx * ny values per plane."""
    case = inputs.three_component(nx=96, ny=192)
    s = Solver(case["params"])
    for C, u, p in ((case["C"][:1], None, None), (case["C"].transpose(0, 2, 1).copy(), None, None),
                    (case["C"], np.zeros((2, 191, 96)), None), (case["C"], None, np.zeros((96, 192)))):
        assert _status(lambda: s.init_fields(0, C, u, p)) == -1
    s.init_fields(0, case["C"])
