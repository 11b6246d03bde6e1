"""Host logic of the checkpointed adjoint driver, run on the CPU against a
stand-in lattice whose "state" is the number of steps taken: the forward
interval reaches the right state without touching its source or copying a
state, and the reverse schedule covers every step of an interval once,
latest first."""
import pytest

from paper_2208_05429_amd.adjoint import forward_interval, reverse_schedule


class Box:
    """A state buffer: the step count it holds."""

    def __init__(self, t=None):
        self.t = t


class CountingLattice:
    def __init__(self):
        self.f = Box()
        self.passes = []  # (k, out_of_place)

    def step_into(self, src, dst, k):
        assert k in (1, 2) and src is not dst and src.t is not None
        dst.t = src.t + k
        self.passes.append((k, True))

    def step(self, n):
        assert n >= 1 and self.f.t is not None
        self.f.t += n
        self.passes.append((n, False))


@pytest.mark.parametrize("n", range(1, 12))
@pytest.mark.parametrize("final", [False, True])
def test_forward_interval_reaches_the_state_without_copies(n, final):
    lat = CountingLattice()
    src = Box(100)
    dst = None if final else Box()
    forward_interval(lat, src, dst, n)
    out = lat.f if final else dst
    assert out.t == 100 + n
    assert src.t == 100  # the kept state at the interval start is untouched
    assert sum(k for k, _ in lat.passes) == n
    # out-of-place passes only at the ends of the interval, one or two steps each
    oop = [i for i, (_, o) in enumerate(lat.passes) if o]
    assert oop[0] == 0 and all(lat.passes[i][0] <= 2 for i in oop)
    if not final:
        assert oop[-1] == len(lat.passes) - 1
    assert len(oop) <= 2


@pytest.mark.parametrize("n", range(1, 12))
@pytest.mark.parametrize("merged", [False, True])
def test_reverse_schedule_covers_each_step_once_latest_first(n, merged):
    calls = reverse_schedule(n, merged)
    covered = [t for t0, k in calls for t in range(t0, t0 + k)]
    assert sorted(covered) == list(range(n))
    assert [t0 for t0, _ in calls] == sorted((t0 for t0, _ in calls), reverse=True)
    assert all(k == (2 if merged else 1) for _, k in calls[:-1])
    if merged:
        # only every other state is needed
        assert len({t0 for t0, _ in calls}) == (n + 1) // 2
