"""Lockstep comparison of the HIP library with the FP64 oracle.

Protocol: at each compared tick the oracle takes the GPU's state (positions,
tick index), computes the FP64 field P_t and the tick's outcome, and the two
are compared:
  * field: the GPU's FP32 field must be the oracle's FP64 field rounded to
    FP32, bit for bit, on every su (both sides sum FP32 strengths exactly in
    FP64 and round once); the relative error max |P_gpu - P_oracle| /
    max(|P_oracle|, 1) over non-obstacle su, at most 2^-24, is reported
    beside it against the 1e-5 bound;
  * per pedestrian: chosen su, election result and new position must match
    bit for bit.  Mismatches are classified: "tied" where the oracle flags a
    near tie (its two best FP64 candidate values within 1e-5 relative) or the
    mismatch is caused by one (a near-tied pedestrian whose oracle or GPU
    target equals this pedestrian's target, either side's, or its position),
    "untied" otherwise.  With a bit-exact field both sides take every FP32
    decision on the same numbers, so neither kind may occur.
"""
from __future__ import annotations

import numpy as np

import oracle

FIELD_RTOL = 1e-5
# threads of the oracle's field (the same bits as one thread)
THREADS = min(16, oracle.host_threads())


def assert_parity(rep: "Report"):
    """The bar: a bit-exact field and no mismatched decision of either kind."""
    assert rep.field_mismatch == 0, rep
    assert rep.max_field_err <= FIELD_RTOL, rep
    assert rep.untied == 0, (rep, rep.first_untied)
    assert rep.tied_mismatch == 0, rep


def field_bits_differ(P_gpu: np.ndarray, P_orc: np.ndarray) -> int:
    """Number of su whose GPU value is not the oracle's FP64 value rounded to
    FP32 (+inf on obstacles on both sides)."""
    return int(np.count_nonzero(np.asarray(P_gpu, np.float32) != P_orc.astype(np.float32)))


def field_rel_err(P_gpu: np.ndarray, P_orc: np.ndarray, obstacle: np.ndarray) -> float:
    free = obstacle == 0
    a = P_gpu[free].astype(np.float64)
    b = P_orc[free]
    if a.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1.0)))


def classify(pos_before, r: "oracle.StepResult", tgt_g, flags_g, pos_g):
    """(untied mismatch ids, tied mismatch ids)."""
    from paper_1803_04782_amd.sf import SF_FLAG_WON

    live = pos_before >= 0
    won_g = (flags_g & SF_FLAG_WON) != 0
    tgt_o = np.where(live, r.target, -1)
    tgt_gg = np.where(live, tgt_g, -1)
    bad = live & ((tgt_o != tgt_gg) | (won_g != (r.moved == 1)) | (pos_g != r.pos))
    if not bad.any():
        return np.array([], np.int64), np.array([], np.int64)
    tied = np.flatnonzero(live & (r.tied == 1))
    hot = set(np.concatenate([r.target[tied], tgt_g[tied]]).tolist())
    untied, tie = [], []
    for j in np.flatnonzero(bad):
        if r.tied[j] or tgt_o[j] in hot or tgt_gg[j] in hot or pos_before[j] in hot:
            tie.append(j)
        else:
            untied.append(j)
    return np.array(untied, np.int64), np.array(tie, np.int64)


class Report:
    def __init__(self):
        self.steps = 0
        self.max_field_err = 0.0
        self.field_mismatch = 0
        self.untied = 0
        self.tied_mismatch = 0
        self.tied_flags = 0
        self.decisions = 0
        self.first_untied = None

    def __repr__(self):
        return (f"Report(steps={self.steps}, max_field_err={self.max_field_err:.3g}, "
                f"field_mismatch={self.field_mismatch}, "
                f"untied={self.untied}, tied_mismatch={self.tied_mismatch}, "
                f"tied_flags={self.tied_flags}, decisions={self.decisions})")


def compare_tick(g, st, report: Report, t: int):
    """Compare one tick of GPU scene `g` (about to run tick t) with the oracle."""
    pos = g.positions()
    P_gpu = g.field()
    r = oracle.step(st, pos, t, threads=THREADS)
    err = field_rel_err(P_gpu, r.P, st.obstacle)
    report.field_mismatch += field_bits_differ(P_gpu, r.P)
    g.step(1)
    tgt_g, flags_g = g.last_moves()
    pos_g = g.positions()
    untied, tied = classify(pos, r, tgt_g, flags_g, pos_g)
    report.steps += 1
    report.max_field_err = max(report.max_field_err, err)
    report.untied += len(untied)
    report.tied_mismatch += len(tied)
    report.tied_flags += int(r.tied[pos >= 0].sum())
    report.decisions += int((pos >= 0).sum())
    if len(untied) and report.first_untied is None:
        j = int(untied[0])
        report.first_untied = dict(t=t, id=j, pos=int(pos[j]), tgt_orc=int(r.target[j]),
                                   tgt_gpu=int(tgt_g[j]), moved_orc=int(r.moved[j]),
                                   flags_gpu=int(flags_g[j]), pos_orc=int(r.pos[j]),
                                   pos_gpu=int(pos_g[j]))
    return r


def lockstep(g, st, t0: int, n_steps: int, every: int = 1) -> Report:
    rep = Report()
    t = t0
    done = 0
    while done < n_steps:
        if done % every == 0:
            compare_tick(g, st, rep, t)
        else:
            g.step(1)
        t += 1
        done += 1
    return rep


def tie_nearby(st, occ, owner, targets) -> bool:
    """True if a registrant of one of `targets` is near-tied (cascade)."""
    W, H = st.W, st.H
    for q in targets:
        qx, qy = q % W, q // W
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                x, y = qx + dx, qy + dy
                if st.periodic:
                    x, y = x % W, y % H
                if (dx or dy) and 0 <= x < W and 0 <= y < H and owner[y * W + x] >= 0:
                    j = int(owner[y * W + x])
                    if oracle.decide_at(st, occ, y * W + x, st.heading_of(j))[1]:
                        return True
    return False


def sampled_field_err(st, obstacle, pos, P_gpu, cells) -> float:
    """Max relative field error at sampled su from the oracle's point route."""
    occ = oracle.occupancy(st.W, st.H, pos)
    ref = oracle.field_at(st, occ, cells)
    free = obstacle[cells] == 0
    if not free.any():
        return 0.0
    return float(np.max(np.abs(P_gpu[cells][free] - ref[free]) /
                        np.maximum(np.abs(ref[free]), 1.0)))


def sampled_outcomes(st, exit_mask, pos, t, ids, tgt_g, flags_g, pos_g):
    """Untied mismatches among pedestrians `ids` for the tick from positions
    `pos` at tick t, against the oracle's point route (target, election,
    exit).  Each entry: (id, oracle target, GPU target, oracle moved, GPU won)."""
    from paper_1803_04782_amd.sf import SF_FLAG_WON

    occ = oracle.occupancy(st.W, st.H, pos)
    live = np.flatnonzero(pos >= 0)
    owner = np.full(st.W * st.H, -1, np.int64)
    owner[pos[live]] = live
    bad = []
    for i in ids:
        tgt, moved, tied = oracle.outcome_at(st, occ, owner, pos, int(i), t)
        won_g = bool(flags_g[i] & SF_FLAG_WON)
        same = tgt == tgt_g[i] and moved == won_g and (
            pos_g[i] == (-1 if moved and exit_mask[tgt] else (tgt if moved else pos[i])))
        if not same and not tied and not tie_nearby(st, occ, owner, (tgt, int(tgt_g[i]))):
            bad.append((int(i), tgt, int(tgt_g[i]), moved, won_g))
    return bad
