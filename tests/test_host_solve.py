"""Host logic of the steady-state orchestration (warmstart.run_to_tolerance)
on a scripted stand-in for the C ABI: no GPU.  Each scripted channel has a
residual history r(step); the stand-in retires a channel at the first
check with r <= tol, as lbm_solve does.

Checked: a channel that converges in float32 is left alone; a channel whose
float32 residual levels off (or falls less than fourfold per 100 000 steps
below 1e-7) moves to float64, its state is written back, it is retired from
the float32 context and its record carries the total steps; nothing is done
past the step cap; float64 contexts are never finished again; a channel
whose state turns non-finite is started again from rest once (lbm_restart),
keeps its steps, and is reported diverged if it diverges again."""
import numpy as np
import pytest

from paper_2210_07501_amd import warmstart as ws


class FakeCtx:
    def __init__(self, hist, prec, owner):
        self.hist = hist            # per channel: function steps -> r
        self.prec = prec
        self.steps = [0] * len(hist)
        self.retired = [None] * len(hist)
        self.bad = [False] * len(hist)
        self.owner = owner


class FakeLBM:
    """Scripted stand-in for the binding: float32 channels follow their
    scripted residual; a float64 context converges after `fp64_steps`."""
    LBM_FP64, LBM_FP32_DEV = 0, 1
    LBM_OK, LBM_EDIVERGED = 0, -4

    class LBMError(RuntimeError):
        def __init__(self, status, where):
            super().__init__("%s: %d" % (where, status))

    def __init__(self, hist, fp64_steps=20_000):
        self.hist = hist
        self.fp64_steps = fp64_steps
        self.calls = []

    def lbm_create(self, cfgs, precision=0):
        hist = [self.hist[c["id"]] if precision == self.LBM_FP32_DEV else (lambda s: 1e-6 if s < self.fp64_steps else 1e-9)
                for c in cfgs]
        self.calls.append(("create", precision, [c["id"] for c in cfgs]))
        ctx = FakeCtx(hist, precision, self)
        ctx.names = [c["id"] for c in cfgs]
        return ctx

    def _r(self, ctx, k):
        return ctx.hist[k](ctx.steps[k]) if ctx.steps[k] > 0 else np.inf

    def lbm_solve(self, ctx, tol, n):
        for k in range(len(ctx.hist)):
            if ctx.retired[k] is not None:
                continue
            for s in range(100, n + 1, 100):       # checks every 100 steps
                ctx.steps[k] += 100
                r = self._r(ctx, k)
                if np.isnan(r):                    # the check kernel's non-finite flag
                    ctx.bad[k] = True
                    ctx.retired[k] = ctx.steps[k]
                    break
                if r <= tol:
                    ctx.retired[k] = ctx.steps[k]
                    break
        active = sum(r is None for r in ctx.retired)
        return (self.LBM_EDIVERGED if any(ctx.bad) else self.LBM_OK), active

    def lbm_residual(self, ctx, k):
        return dict(r=self._r(ctx, k), steps=ctx.steps[k], sum_phi=0.0, sum_mass=0.0, u_int_peak=0.0,
                    diverged=ctx.bad[k])

    def lbm_restart(self, ctx, k, fields=None):
        """Cold start of channel k at the current step: its script restarts
        from rest (the "after_restart" history of the channel, if any)."""
        self.calls.append(("restart", ctx.prec, k))
        assert fields is None
        at = ctx.steps[k]
        after = AFTER_RESTART[ctx.names[k]]
        ctx.hist[k] = (lambda a, f: (lambda s: f(s - a)))(at, after)
        ctx.bad[k] = False
        ctx.retired[k] = None

    def lbm_get_state(self, ctx, k):
        self.calls.append(("get", ctx.prec, k))
        return np.full((3, 9, 2, 2), float(k))

    def lbm_set_state(self, ctx, k, pop):
        self.calls.append(("set", ctx.prec, k))

    def lbm_retire(self, ctx, k):
        self.calls.append(("retire", ctx.prec, k))
        ctx.retired[k] = ctx.steps[k]

    def lbm_destroy(self, ctx):
        pass


def _converges(s):
    return 1e-5 * np.exp(-s / 20_000.0)                                       # < 1e-8 near 138 000


# residual history after a cold restart (lbm_restart) of each scripted channel
AFTER_RESTART = {"nan_start": _converges, "nan_twice": lambda s: np.nan}


def scripted():
    return {
        "nan_start": lambda s: np.nan,                                         # a non-finite warm start
        "nan_twice": lambda s: np.nan,                                         # diverges from rest too
        "converges": _converges,
        "floor": lambda s: max(1e-5 * np.exp(-s / 20_000.0), 2.5e-8),            # levels off at 2.5e-8
        "slow": lambda s: max(1e-5 * np.exp(-s / 30_000.0), 5e-8 * np.exp(-s / 400_000.0)),  # tail too slow
    }


def run(names, cap, prec=FakeLBM.LBM_FP32_DEV, monkeypatch=None):
    fake = FakeLBM(scripted())
    monkeypatch.setattr(ws, "lbm", fake)
    cfgs = [dict(id=n) for n in names]
    ctx = fake.lbm_create(cfgs, precision=prec)
    res = ws.run_to_tolerance(ctx, cfgs, prec, tol=1e-8, cap=cap, chunk=50_000, verbose=False)
    return fake, ctx, res


def test_converging_channel_is_left_alone(monkeypatch):
    fake, ctx, res = run(["converges"], 400_000, monkeypatch=monkeypatch)
    assert res[0]["r"] <= 1e-8 and not res[0].get("finished_fp64")
    assert not any(c[0] == "retire" for c in fake.calls)


def test_floor_and_slow_tail_are_finished_in_float64(monkeypatch):
    fake, ctx, res = run(["converges", "floor", "slow"], 600_000, monkeypatch=monkeypatch)
    assert not res[0].get("finished_fp64")
    for k in (1, 2):
        assert res[k]["finished_fp64"] and res[k]["r"] <= 1e-8
        # float32 steps up to the detection, then the float64 steps
        assert res[k]["steps"] == ctx.steps[k] + fake.fp64_steps
        assert ("retire", FakeLBM.LBM_FP32_DEV, k) in fake.calls
        assert ("set", FakeLBM.LBM_FP32_DEV, k) in fake.calls      # finished state written back
    # a float64 context was created for the finished channels only
    created = [c for c in fake.calls if c[0] == "create" and c[1] == FakeLBM.LBM_FP64]
    assert created and all(set(c[2]) <= {"floor", "slow"} for c in created)
    assert all(s <= 600_000 for s in ctx.steps)


def test_nothing_is_finished_past_the_cap(monkeypatch):
    # the floor cannot be detected within 150 000 steps (two checks 100 000 apart needed)
    fake, ctx, res = run(["floor"], 150_000, monkeypatch=monkeypatch)
    assert not res[0].get("finished_fp64") and res[0]["r"] > 1e-8
    assert max(ctx.steps) <= 150_000


def test_float64_contexts_are_not_finished_again(monkeypatch):
    fake, ctx, res = run(["floor"], 400_000, prec=FakeLBM.LBM_FP64, monkeypatch=monkeypatch)
    assert not any(c[0] in ("retire", "get") for c in fake.calls)


def test_diverged_channel_restarts_from_rest(monkeypatch):
    fake, ctx, res = run(["converges", "nan_start"], 400_000, monkeypatch=monkeypatch)
    assert not res[0]["restarted_cold"] and res[0]["r"] <= 1e-8
    assert res[1]["restarted_cold"] and not res[1]["diverged"] and res[1]["r"] <= 1e-8
    # it diverged at its first check (step 100, inside the first 50 000-step
    # chunk), was restarted at that step and charged those 100 steps too
    assert ("restart", FakeLBM.LBM_FP32_DEV, 1) in fake.calls
    assert res[1]["steps"] == 100 + 138_200
    assert sum(c[0] == "restart" for c in fake.calls) == 1


def test_channel_diverging_from_rest_is_reported_not_restarted_again(monkeypatch):
    fake, ctx, res = run(["nan_twice", "converges"], 400_000, monkeypatch=monkeypatch)
    assert res[0]["restarted_cold"] and res[0]["diverged"]
    assert sum(c[0] == "restart" for c in fake.calls) == 1
    assert res[1]["r"] <= 1e-8


def test_training_refuses_an_empty_set():
    """No converged channel (or fewer than one batch): a clear error before
    any network call, not a division by zero after the first epoch."""
    import torch
    from paper_2210_07501_amd import warmstart as ws
    X = torch.empty((3, 4, 64, 32), dtype=torch.bfloat16)
    Y = torch.empty((3, 4, 64, 4))
    with pytest.raises(ValueError, match="at least one batch"):
        ws.train(None, X, Y, epochs=1, batch=16)
