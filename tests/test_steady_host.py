"""Host logic of the batched time-to-steady arms (no GPU): the window loop of
steady.batch_arm with the warm start, against a stand-in batch whose cases
converge, stall or diverge at set step counts.  Checks the bookkeeping of the
cold-start fallback: a warm-started case that diverges is reset to rest in
the batch, runs the filter again with a full step budget, and its steps
count the failed attempt."""
import numpy as np
import pytest

from workloads import Case

# per case: steps from rest to convergence (None: never), steps from the
# prediction to convergence, step at which the prediction diverges
COLD_CONV = [5000, 30000, None, 4000]
WARM_CONV = [4000, None, None, 3000]
WARM_DIV = [None, 100, None, None]


class FakeBatch:
    def __init__(self, grids, masks, params):
        self.n = len(grids)
        self.mode = ["cold"] * self.n
        self.age = np.zeros(self.n, np.int64)
        self.st = np.zeros(self.n, np.int32)
        self.enabled = np.ones(self.n, np.int32)
        self.restarts = 0

    def set_launch(self, *a):
        pass

    def init_fields_device(self, j, *p):
        self.mode[j], self.age[j] = "warm", 0

    def init_fields(self, j, *a):
        assert all(x is None for x in a)
        self.mode[j], self.age[j] = "cold", 0
        self.restarts += 1

    def set_enabled(self, e=None):
        self.enabled = np.ones(self.n, np.int32) if e is None else np.asarray(e, np.int32)

    def set_plateau(self, *a):
        pass

    def average_last_two(self):
        pass

    def run(self, tol, m):
        steps = np.zeros(self.n, np.int64)
        self.st[:] = 0
        for i in range(self.n):
            if not self.enabled[i]:
                continue
            if self.mode[i] == "nan":
                self.st[i], steps[i] = 3, -100
                continue
            warm = self.mode[i] == "warm"
            div = WARM_DIV[i] if warm else None
            conv = (WARM_CONV if warm else COLD_CONV)[i]
            if div is not None and self.age[i] + m >= div:
                steps[i], self.st[i] = -(div - self.age[i]), 3
                self.age[i], self.mode[i] = div, "nan"
            elif tol > 0 and conv is not None and self.age[i] + m >= conv:
                steps[i], self.st[i] = conv - self.age[i], 1
                self.age[i] = conv
            else:
                steps[i] = m
                self.age[i] += m
        return steps

    def status(self):
        return self.st.copy()

    def fields(self, i, ny, nx):
        mark = {"cold": 1.0, "warm": 2.0, "nan": np.nan}[self.mode[i]]
        return np.ones((ny, nx)), np.full((ny, nx), mark), np.zeros((ny, nx))

    def close(self):
        pass


class Net:
    kinds = ("cavity",)


@pytest.fixture
def arm(monkeypatch):
    import torch
    from paper_1806_10251_amd import steady, surrogate
    made = []

    def batch(*a):
        made.append(FakeBatch(*a))
        return made[-1]
    monkeypatch.setattr(steady.L, "Batch", batch)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a: None)
    monkeypatch.setattr(surrogate, "predict_fields",
                        lambda net, cases: [("p",) if surrogate.covers(k, net) else None
                                            for k in cases])
    cases = [Case("cavity", 16, 16, 100.0, 0.5, 0.1, np.zeros((16, 16), np.uint8))
             for _ in COLD_CONV]

    def run(warm, max_steps=50_000, segment=None):
        out = steady.batch_arm(cases, 1e-8, max_steps, "f64", None,
                               Net() if warm else None, surrogate.WARM_FILTER,
                               segment=segment)
        return out, made[-1]
    return run


def test_cold_arm_steps_and_status(arm):
    (steps, st, _, fields), _ = arm(False)
    assert list(st) == [1, 1, 0, 1]
    assert list(steps) == [5000, 30000, 50000, 4000]


def test_warm_arm_resets_a_diverged_prediction_in_the_batch(arm):
    (steps, st, _, fields), b = arm(True)
    assert b.restarts == 1
    assert list(st) == [1, 1, 0, 1]
    # case 1: the prediction diverged inside the filter steps (1000 steps
    # counted), then the cold run from rest (30000 steps, filter included)
    assert steps[1] == 1000 + 30000
    assert list(steps[[0, 2, 3]]) == [4000, 50000, 3000]
    assert fields[1][0][0, 0] == 1.0 and fields[0][0][0, 0] == 2.0


def test_fallback_gets_a_full_budget_and_windows_respect_each_limit(arm):
    (steps, st, _, _), _ = arm(True, max_steps=20_000, segment=3000)
    # case 1 never converges within its own 20000-step budget after the reset
    assert st[1] == 0 and steps[1] == 1000 + 20_000
    assert st[2] == 0 and steps[2] == 20_000
    assert list(st[[0, 3]]) == [1, 1] and list(steps[[0, 3]]) == [4000, 3000]
