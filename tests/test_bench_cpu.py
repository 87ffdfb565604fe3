"""Host logic of the benchmark script: the warm-up that makes a timed call
replay a captured graph, and the code hash that keys the traffic record."""
import bench


class FakeSim:
    """Counts steps like the library and records each call's starting
    (re-sort phase, state-buffer parity), the key of a graph capture."""

    def __init__(self, R, start=0):
        self.R, self.g, self.keys = R, start, []

    def stats(self):
        return {"reorder_every": self.R, "steps_total": self.g}

    def key(self):
        if self.R <= 0:
            return (0, 0)
        reorders = sum(1 for k in range(self.g) if k % self.R == 0)   # swaps so far
        return (self.g % self.R, reorders % 2)

    def step(self, k):
        self.keys.append(self.key())
        self.g += k


def test_replay_ready_ends_where_the_next_call_repeats_a_captured_key():
    for R, steps, start in ((8, 100, 0), (32, 100, 400), (16, 96, 10), (16, 5, 37), (32, 1, 0), (0, 100, 0)):
        sim = FakeSim(R, start)
        made = bench.replay_ready(sim, steps, sim.step)
        assert made == steps * len(sim.keys)
        assert sim.key() in sim.keys, (R, steps, start)          # the timed call replays
        assert len(set(sim.keys)) == len(sim.keys)               # no call wasted on a seen key


def test_code_hash_ignores_comments_and_layout():
    a = "int f(int x) {  // the answer\n  return x + 1;\n}\n"
    b = "int f(int x) {\n    return x + 1;   // same code\n}\n"
    c = "int f(int x) {\n  return x + 2;\n}\n"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)
    assert len(bench.kernel_source_hash()) == 16
