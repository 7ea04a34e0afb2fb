"""Autotuner of the batched plans' kernel variants.

The library exposes tuning knobs (``fm_set_knob`` in include/fastmusic.h):
for a shape bucket, a knob picks one of several kernel variants that all
compute bit-identical results and differ only in speed.  ``tune`` times every
variant of every knob on the caller's own frames -- for each bucket present
in the batch, a plan over (up to ``max_frames``) frames of that bucket, the
one stage the knob affects, timed with HIP events on the launch stream,
median of ``reps`` -- and installs the fastest on the context.  Results go to
a JSON cache keyed by device, library build and precision, so a later run
with the same shapes installs them without timing (``apply``).

Knobs and buckets:
  cov_schedule   bucket log2(M) - 7 in [0, 5]; 0 = a frame's covariance tiles
                 on one XCD, 1 = tiles dealt one by one to the XCDs (the
                 built-in 2 picks per precision; tuning installs 0 or 1)
  spec_angles    bucket ceil(K/8) - 1 in [0, 7]; angles per workgroup of the
                 FP32 (polynomial) spectrum pass, which every plan runs (64,
                 128, 256 for buckets 0..3)
  spec16_angles  the same for the compensated FP16 pass (single-frame calls)
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from dataclasses import dataclass, field

from . import (FM_FP32, FM_KNOB_COV_SCHEDULE, FM_KNOB_SPEC16_ANGLES, FM_KNOB_SPEC_ANGLES,
               LIB_PATH)

KNOB_NAMES = {FM_KNOB_COV_SCHEDULE: "cov_schedule", FM_KNOB_SPEC_ANGLES: "spec_angles",
              FM_KNOB_SPEC16_ANGLES: "spec16_angles"}
# the plan stage each knob changes
KNOB_STAGE = {FM_KNOB_COV_SCHEDULE: "covariance", FM_KNOB_SPEC_ANGLES: "pseudospectrum",
              FM_KNOB_SPEC16_ANGLES: "pseudospectrum"}


def cov_bucket(M: int) -> int:
    b = 0
    while b < 5 and (128 << b) < M:
        b += 1
    return b


def spec_bucket(K: int) -> int:
    return (K + 7) // 8 - 1


def bucket_of(knob: int, M: int, K: int) -> int:
    return cov_bucket(M) if knob == FM_KNOB_COV_SCHEDULE else spec_bucket(K)


def choices(knob: int, bucket: int) -> list[int]:
    if knob == FM_KNOB_COV_SCHEDULE:
        return [0, 1]
    return [64, 128, 256] if bucket < 4 else [64, 128]


def knobs_for(prec: int) -> list[int]:
    """Knobs that affect a plan at precision `prec` (every plan runs the FP32
    polynomial spectrum pass; the FP16 pass knob only affects single-frame
    fm_pseudospectrum calls at FM_FP16)."""
    return [FM_KNOB_COV_SCHEDULE, FM_KNOB_SPEC_ANGLES]


@dataclass
class Choice:
    value: int
    ms: dict = field(default_factory=dict)   # variant -> median ms
    frames: int = 0


def _median(xs):
    xs = sorted(xs)
    n = len(xs)
    return xs[n // 2] if n % 2 else 0.5 * (xs[n // 2 - 1] + xs[n // 2])


def _time_stage_events(plan, stage: str, reps: int, stream) -> float:
    """Median ms of one plan stage over `reps` launches (HIP events on the
    launch stream, after one untimed launch)."""
    import torch
    run = getattr(plan, stage)
    run(stream)
    out = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        run(stream)
        e1.record(stream)
        e1.synchronize()
        out.append(e0.elapsed_time(e1))
    return _median(out)


def tune(ctx, frames, prec: int = FM_FP32, reps: int = 5, max_frames: int = 64,
         knobs=None, make_plan=None, time_stage=None, stream=None, log=None) -> dict:
    """Times every variant of each knob on the frames of each bucket and
    installs the fastest on `ctx`.

    frames: objects with ``spec.M``, ``spec.K`` and ``descriptor()`` (the
    frames' buffers must already hold a computed subspace, e.g. after one
    ``Plan.run()``, so the spectrum stage sees realistic data).
    make_plan(ctx, descriptors, prec) and time_stage(plan, stage, reps)
    default to ``Plan`` and HIP-event timing.  Returns
    {knob: {bucket: Choice}}.
    """
    if make_plan is None:
        from . import Plan

        def make_plan(c, descs, p):
            return Plan(c, descs, prec=p)
    if time_stage is None:
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()

        def time_stage(plan, stage, r):
            return _time_stage_events(plan, stage, r, s)
    table: dict = {}
    for knob in (knobs if knobs is not None else knobs_for(prec)):
        groups: dict[int, list] = {}
        for fr in frames:
            groups.setdefault(bucket_of(knob, fr.spec.M, fr.spec.K), []).append(fr)
        table[knob] = {}
        for bucket in sorted(groups):
            sub = groups[bucket][:max_frames]
            descs = [f.descriptor() for f in sub]
            keep = ctx.get_knob(knob, bucket)
            res = Choice(value=keep, frames=len(sub))
            for v in choices(knob, bucket):
                ctx.set_knob(knob, bucket, v)
                plan = make_plan(ctx, descs, prec)
                try:
                    res.ms[v] = float(time_stage(plan, KNOB_STAGE[knob], reps))
                finally:
                    plan.close()
            res.value = min(res.ms, key=lambda v: (res.ms[v], v))
            ctx.set_knob(knob, bucket, res.value)
            table[knob][bucket] = res
            if log:
                log(f"tune {KNOB_NAMES[knob]} bucket {bucket} ({len(sub)} frames): "
                    + ", ".join(f"{v}: {t:.3f} ms" for v, t in res.ms.items())
                    + f" -> {res.value}")
    return table


def apply(ctx, table: dict) -> None:
    """Installs a table from ``tune`` or ``load`` on a context."""
    for knob, per in table.items():
        for bucket, ch in per.items():
            ctx.set_knob(int(knob), int(bucket), int(ch.value))


def library_id(path: str = LIB_PATH) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def cache_key(device_name: str, lib_id: str, prec: int) -> str:
    return f"{device_name}|{lib_id}|prec{prec}"


def to_json(table: dict) -> dict:
    return {KNOB_NAMES[k]: {str(b): {"value": c.value, "frames": c.frames,
                                     "ms": {str(v): round(t, 5) for v, t in c.ms.items()}}
                            for b, c in per.items()}
            for k, per in table.items()}


def from_json(obj: dict) -> dict:
    by_name = {v: k for k, v in KNOB_NAMES.items()}
    out: dict = {}
    for name, per in obj.items():
        knob = by_name[name]
        out[knob] = {int(b): Choice(value=int(c["value"]), frames=int(c.get("frames", 0)),
                                    ms={int(v): float(t) for v, t in c.get("ms", {}).items()})
                     for b, c in per.items()}
    return out


def save(path: str, key: str, table: dict) -> None:
    """Adds (or replaces) one entry of the JSON cache at `path`."""
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[key] = {"saved": time.strftime("%Y-%m-%dT%H:%M:%S"), "knobs": to_json(table)}
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def load(path: str, key: str) -> dict | None:
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    ent = data.get(key)
    return None if ent is None else from_json(ent["knobs"])
