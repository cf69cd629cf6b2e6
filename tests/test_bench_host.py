"""bench.py's host-side decisions, with stand-in objects (no GPU)."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


class _Lib:
    MAP_ADDS_AUTO, MAP_ADDS_64, MAP_ADDS_32 = 0, 1, 2


class _Sim:
    """Kernel time per run as a function of the map-add kind in force."""

    def __init__(self, ms_by_kind):
        self.ms_by_kind = ms_by_kind
        self.kind = None
        self.runs = []

    def set_map_adds(self, kind):
        self.kind = kind

    def run(self, n, seed):
        self.runs.append((self.kind, n, seed))

    def stats(self):
        return {"kernel_ms": self.ms_by_kind[self.kind]}


def test_map_adds_keeps_the_faster_kind_at_full_size():
    b = _bench()
    for ms, want in [({2: 512.3, 1: 547.1}, 2), ({2: 820.0, 1: 760.0}, 1)]:
        sim = _Sim(ms)
        note = b.map_adds_at_full_size(_Lib, sim, 100_000_000, 7)
        assert sim.kind == want  # left in force for the timed steps
        # one run of each kind, at the full photon count
        assert sorted(k for k, _, _ in sim.runs) == [1, 2]
        assert all(n == 100_000_000 for _, n, _ in sim.runs)
        assert f"{ms[2]:.1f} ms" in note and f"{ms[1]:.1f} ms" in note
