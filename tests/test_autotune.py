"""Host logic of the autotuner: bucketing, variant sets, argmin selection,
installation on the context and the JSON cache (fake context, plans and
timer; no GPU)."""
import pytest

import paper_1911_07434_amd as fm
from paper_1911_07434_amd import autotune as at


class FakeCtx:
    def __init__(self):
        self.knobs = {}

    def set_knob(self, k, b, v):
        assert v in at.choices(k, b)
        self.knobs[(k, b)] = v

    def get_knob(self, k, b):
        return self.knobs.get((k, b), at.choices(k, b)[0])


class Spec:
    def __init__(self, M, K):
        self.M, self.K = M, K


class Frame:
    def __init__(self, M, K):
        self.spec = Spec(M, K)

    def descriptor(self):
        return (self.spec.M, self.spec.K)


class FakePlan:
    def __init__(self, ctx, descs, prec):
        self.snapshot = dict(ctx.knobs)   # the knob values the plan was built with
        self.descs = descs
        self.closed = False

    def close(self):
        self.closed = True


def test_buckets_and_choices():
    assert [at.cov_bucket(M) for M in (64, 128, 129, 256, 1024, 2048, 4096, 8192)] == \
        [0, 0, 1, 1, 3, 4, 5, 5]
    assert [at.spec_bucket(K) for K in (1, 8, 9, 16, 17, 64)] == [0, 0, 1, 1, 2, 7]
    assert at.choices(fm.FM_KNOB_COV_SCHEDULE, 3) == [0, 1]
    assert at.choices(fm.FM_KNOB_SPEC_ANGLES, 3) == [64, 128, 256]
    assert at.choices(fm.FM_KNOB_SPEC16_ANGLES, 4) == [64, 128]
    assert at.knobs_for(fm.FM_FP32) == [fm.FM_KNOB_COV_SCHEDULE, fm.FM_KNOB_SPEC_ANGLES]
    # every plan runs the FP32 polynomial spectrum pass
    assert at.knobs_for(fm.FM_FP16) == [fm.FM_KNOB_COV_SCHEDULE, fm.FM_KNOB_SPEC_ANGLES]


def test_tune_picks_fastest_variant_per_bucket_and_installs_it():
    ctx = FakeCtx()
    frames = [Frame(M, K) for M, K in [(256, 3), (256, 12), (1024, 8), (2048, 16), (512, 40)]]
    plans = []
    # synthetic cost: the covariance prefers schedule 1 only for M >= 1024; the
    # spectrum prefers 128 angles, except bucket 0 which prefers 256
    def cost(plan, stage, reps):
        plans.append(plan)
        if stage == "covariance":
            (k, b), = [(k, b) for (k, b) in plan.snapshot if k == fm.FM_KNOB_COV_SCHEDULE
                       and b == at.cov_bucket(plan.descs[0][0])]
            v = plan.snapshot[(k, b)]
            return 1.0 + (0.5 if (v == 1) != (b >= 3) else 0.0)
        b = at.spec_bucket(plan.descs[0][1])
        v = plan.snapshot[(fm.FM_KNOB_SPEC_ANGLES, b)]
        best = 256 if b == 0 else 128
        return 1.0 + abs(v - best) / 64.0
    table = at.tune(ctx, frames, fm.FM_FP32, reps=3, make_plan=FakePlan, time_stage=cost)
    cov = table[fm.FM_KNOB_COV_SCHEDULE]
    assert sorted(cov) == [1, 2, 3, 4]                  # buckets present in the batch
    assert {b: c.value for b, c in cov.items()} == {1: 0, 2: 0, 3: 1, 4: 1}
    spec = table[fm.FM_KNOB_SPEC_ANGLES]
    assert {b: c.value for b, c in spec.items()} == {0: 256, 1: 128, 4: 128}
    assert set(spec[0].ms) == {64, 128, 256} and set(spec[4].ms) == {64, 128}
    assert cov[1].frames == 2 and spec[0].frames == 2
    # installed on the context; every plan closed
    assert ctx.get_knob(fm.FM_KNOB_COV_SCHEDULE, 4) == 1
    assert ctx.get_knob(fm.FM_KNOB_SPEC_ANGLES, 0) == 256
    assert all(p.closed for p in plans)


def test_tune_ties_go_to_the_smaller_value_and_max_frames_caps_the_sample():
    ctx = FakeCtx()
    frames = [Frame(512, 4) for _ in range(10)]
    seen = []

    def flat(plan, stage, reps):
        seen.append(len(plan.descs))
        return 2.0
    table = at.tune(ctx, frames, fm.FM_FP16, max_frames=4, make_plan=FakePlan, time_stage=flat)
    assert table[fm.FM_KNOB_COV_SCHEDULE][2].value == 0
    assert table[fm.FM_KNOB_SPEC_ANGLES][0].value == 64
    assert set(seen) == {4}


def test_cache_round_trip_and_apply(tmp_path):
    ctx = FakeCtx()
    table = {fm.FM_KNOB_COV_SCHEDULE: {3: at.Choice(1, {0: 2.0, 1: 1.5}, 7)},
             fm.FM_KNOB_SPEC16_ANGLES: {0: at.Choice(256, {64: 3.0, 128: 2.0, 256: 1.0}, 9)}}
    path = str(tmp_path / "sub" / "tune.json")
    key = at.cache_key("MI355X", "abc", fm.FM_FP16)
    assert at.load(path, key) is None
    at.save(path, key, table)
    at.save(path, at.cache_key("MI355X", "abc", fm.FM_FP32), {})
    back = at.load(path, key)
    assert {k: {b: (c.value, c.ms, c.frames) for b, c in v.items()} for k, v in back.items()} == \
        {k: {b: (c.value, c.ms, c.frames) for b, c in v.items()} for k, v in table.items()}
    at.apply(ctx, back)
    assert ctx.get_knob(fm.FM_KNOB_COV_SCHEDULE, 3) == 1
    assert ctx.get_knob(fm.FM_KNOB_SPEC16_ANGLES, 0) == 256
    assert at.load(path, at.cache_key("MI355X", "other", fm.FM_FP16)) is None


def test_bad_knob_value_rejected_by_fake_context():
    with pytest.raises(AssertionError):
        FakeCtx().set_knob(fm.FM_KNOB_SPEC_ANGLES, 5, 256)
