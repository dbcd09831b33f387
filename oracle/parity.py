"""Full-size parity of a transport against the oracle (test infrastructure
only: used by the tests and by the benchmark's CPU-baseline leg).

The oracle transports a whole workload in worker processes and returns, per
track slot, a digest of what its step log would hold (hash of the touchable
and limiter sequence, record count, fate, sums of step lengths and deposits),
plus per-event and per-touchable deposits.  Another implementation's digests
are compared slot by slot; every slot that differs is transported again with
full logs on both sides, and the first record where the histories part is
located.  The oracle logs, with every record, the smallest margin |a - b| /
scale of the decisions behind it; a divergence at a decision whose margin is
below FLIP_MARGIN (256 units in the last place of the decision's scale) is a
rounding-edge flip, any other divergence a bug.
"""
from __future__ import annotations

import multiprocessing as mp

import numpy as np

from . import DIGEST_DTYPE, Geometry

FLIP_MARGIN = 256 * 2.0 ** -52
RTOL = 1e-9
ATOL = 1e-12

_JOB = None


def _work(bounds):
    desc, prim, seed, ecut, n_events = _JOB
    lo, hi = bounds
    og = Geometry(desc)
    sub = prim.subset(np.arange(lo, hi))
    r = og.transport(sub, seed=seed, ecut=ecut, n_events=n_events, want_digest=True)
    return lo, r["digest"], r["edep_event"], r["escaped_event"], r["edep_touchable"], r["counters"]


def oracle_run(desc, prim, seed=0, ecut=1e-3, n_events=None, workers=16):
    """Digests [3 n], event deposits and escapes, touchable deposits and counters of the
    oracle over all primaries, in `workers` forked processes (contiguous slices)."""
    global _JOB
    n = prim.n
    ne = prim.n_events if n_events is None else n_events
    _JOB = (desc, prim, seed, ecut, ne)
    cuts = np.linspace(0, n, max(1, workers) + 1).astype(int)
    parts = [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    try:
        if workers > 1 and len(parts) > 1:
            with mp.get_context("fork").Pool(len(parts)) as pool:
                res = pool.map(_work, parts)
        else:
            res = [_work(p) for p in parts]
    finally:
        _JOB = None
    digest = np.zeros(3 * n, DIGEST_DTYPE)
    edep_ev = np.zeros(ne)
    esc_ev = np.zeros(ne)
    edep_t = None
    counters = None
    for lo, d, ee, es, et, c in res:
        digest[3 * lo: 3 * lo + len(d)] = d
        edep_ev += ee
        esc_ev += es
        edep_t = et if edep_t is None else edep_t + et
        counters = dict(c) if counters is None else {k: counters[k] + c[k] for k in counters}
    return dict(digest=digest, edep_event=edep_ev, escaped_event=esc_ev, edep_touchable=edep_t,
                counters=counters)


def digest_mismatches(got, ref):
    """Slots whose digests differ: hash, count or fate unequal, or the sums beyond
    RTOL (relative) + ATOL."""
    bad = (got["hash"] != ref["hash"]) | (got["n"] != ref["n"]) | (got["fate"] != ref["fate"])
    for f in ("sum_step", "sum_edep"):
        a, b = got[f], ref[f]
        bad |= ~(np.abs(a - b) <= RTOL * np.maximum(np.abs(a), np.abs(b)) + ATOL)
    return np.nonzero(bad)[0]


def first_divergence(rec_a, n_a, fate_a, rec_b, n_b, fate_b):
    """Index of the first record where two logs of one track part (touchable or code
    unequal, or a length, deposit or energy beyond the tolerance); the shorter log's
    length when one is a prefix of the other; -1 when they agree."""
    k = min(int(n_a), int(n_b), len(rec_a), len(rec_b))
    for i in range(k):
        a, b = rec_a[i], rec_b[i]
        if a["touchable"] != b["touchable"] or a["code"] != b["code"]:
            return i
        for f in ("step", "edep", "energy"):
            x, y = float(a[f]), float(b[f])
            if not abs(x - y) <= RTOL * max(abs(x), abs(y)) + ATOL:
                return i
    if n_a != n_b or fate_a != fate_b:
        return k
    return -1


def classify(slots, gpu_logs, ora_logs):
    """For each mismatching slot: (slot, record index, oracle margin there, 'flip' or
    'bug').  gpu_logs / ora_logs map slot -> (records, n, fate[, margins, tail])."""
    out = []
    for s in slots:
        ga, gn, gf = gpu_logs[s]
        oa, on, of, om, ot = ora_logs[s]
        i = first_divergence(ga, gn, gf, oa, on, of)
        if i < 0:
            out.append((int(s), -1, float("inf"), "none"))
            continue
        m = float(om[i]) if i < min(int(on), len(om)) else float(ot)
        # the decisions behind record i, and those just before it (a relocation
        # at the end of the previous step), may have parted the histories
        if i > 0:
            m = min(m, float(om[i - 1]))
        out.append((int(s), int(i), m, "flip" if m < FLIP_MARGIN else "bug"))
    return out


def oracle_logs(desc, prim, slots, cap, seed=0, ecut=1e-3, n_events=None):
    """Full logs with margins of the oracle for the primaries owning `slots`."""
    prims = np.unique(np.asarray(slots) // 3)
    og = Geometry(desc)
    sub = prim.subset(prims)
    ne = prim.n_events if n_events is None else n_events
    r = og.transport(sub, seed=seed, ecut=ecut, log_cap=cap, n_events=ne, want_margins=True)
    where = {int(p): j for j, p in enumerate(prims)}
    out = {}
    for s in slots:
        j = 3 * where[int(s) // 3] + int(s) % 3
        out[int(s)] = (r["log"][j], int(r["log_n"][j]), int(r["log_fate"][j]), r["margin"][j],
                       float(r["tail_margin"][j]))
    return out, prims


EXACT_COUNTERS = ("steps", "pe", "compton", "pair", "crossings", "escaped", "cutoff", "pushes", "stuck",
                  "truncated", "tracks")


def full_check(desc, prim, gpu_digest, gpu_logs, gpu_tally=None, seed=0, ecut=1e-3, n_events=None,
               workers=16, cap=4096, max_classified=2000):
    """Compare another implementation with the oracle over every track of a workload.

    gpu_digest: its per-track digests [3 n] (DIGEST_DTYPE); gpu_logs(prim_idx) returns its
    full logs (records [3 k][cap], counts [3 k], fates [3 k]) for the primaries prim_idx;
    gpu_tally (optional): its tallies of a run without logging (edep_event, escaped_event,
    edep_touchable, counters), compared event by event.  Returns the counts of tracks,
    mismatching tracks, flips and bugs, the largest tally differences and the
    classification of each mismatch."""
    ref = oracle_run(desc, prim, seed=seed, ecut=ecut, n_events=n_events, workers=workers)
    used = ref["digest"]["fate"] != 0
    mism = digest_mismatches(gpu_digest, ref["digest"])
    out = dict(tracks=int(used.sum()), mismatches=int(len(mism)), flips=0, bugs=0, classified=[])
    if len(mism):
        slots = mism[:max_classified]
        ora, prims = oracle_logs(desc, prim, slots, cap, seed=seed, ecut=ecut, n_events=n_events)
        rec, n, fate = gpu_logs(prims)
        where = {int(p): j for j, p in enumerate(prims)}
        gl = {}
        for s in slots:
            j = 3 * where[int(s) // 3] + int(s) % 3
            gl[int(s)] = (rec[j], int(n[j]), int(fate[j]))
        cls = classify(slots, gl, ora)
        out["classified"] = cls
        out["flips"] = sum(1 for c in cls if c[3] == "flip")
        out["bugs"] = sum(1 for c in cls if c[3] == "bug") + max(0, len(mism) - len(slots))
    if gpu_tally is not None:
        def rel(a, b):
            d = np.abs(a - b) / np.maximum(np.maximum(np.abs(a), np.abs(b)), 1e-300)
            d[(a == b)] = 0.0
            return float(d.max()) if d.size else 0.0
        out["max_rel_event_deposit"] = rel(gpu_tally["edep_event"], ref["edep_event"])
        out["max_rel_event_escape"] = rel(gpu_tally["escaped_event"], ref["escaped_event"])
        et, rt = gpu_tally["edep_touchable"], ref["edep_touchable"]
        out["max_rel_touchable_deposit"] = rel(et, rt)
        out["counters_equal"] = all(gpu_tally["counters"][k] == ref["counters"][k] for k in EXACT_COUNTERS)
    out["oracle_counters"] = ref["counters"]
    return out
