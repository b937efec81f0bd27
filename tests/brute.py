"""Independent brute-force labellers used to pin the oracle (and, on tiny inputs,
the device path).  They share nothing with the oracle's breadth-first search:

* ``propagate_labels`` -- min-label propagation to a fixed point over a stack of
  small binary grids (numpy, vectorised over the stack);
* ``pairwise_components`` -- all-pairs adjacency + union by relabelling, for a
  handful of digis.
"""
from __future__ import annotations

import numpy as np

ROWS, COLS, PIX = 160, 416, 160 * 416


def propagate_labels(fired: np.ndarray) -> np.ndarray:
    """fired: (P, R, C) bool.  Returns (P, R, C) int32 labels: for a fired cell the
    smallest column-major local index ``c*R + r`` in its 8-connected component,
    else -1."""
    P, R, C = fired.shape
    big = R * C
    idx = (np.arange(C)[None, :] * R + np.arange(R)[:, None]).astype(np.int32)
    dt = np.uint8 if big < 255 else np.int32
    lab = np.full((P, R + 2, C + 2), big, dtype=dt)
    lab[:, 1:-1, 1:-1] = np.where(fired, idx[None], big)
    inner = np.zeros((P, R + 2, C + 2), dtype=bool)
    inner[:, 1:-1, 1:-1] = fired
    while True:
        m = lab[:, 1:-1, 1:-1].copy()
        for dr in (0, 1, 2):
            for dc in (0, 1, 2):
                np.minimum(m, lab[:, dr:dr + R, dc:dc + C], out=m)
        m = np.where(fired, m, big).astype(dt)
        if np.array_equal(m, lab[:, 1:-1, 1:-1]):
            break
        lab[:, 1:-1, 1:-1] = m
    out = lab[:, 1:-1, 1:-1].astype(np.int32)
    out[~fired] = -1
    return out


def pairwise_components(module, row, col, adc, cut):
    """O(n^2) reference for tiny events.  Returns (digi ids, [(id, charge, size)] kept,
    ascending)."""
    module = np.asarray(module, np.int64)
    row = np.asarray(row, np.int64)
    col = np.asarray(col, np.int64)
    adc = np.asarray(adc, np.int64)
    n = module.size
    label = list(range(n))
    for i in range(n):
        for j in range(i + 1, n):
            if module[i] == module[j] and abs(row[i] - row[j]) <= 1 and abs(col[i] - col[j]) <= 1:
                a, b = label[i], label[j]
                if a != b:
                    label = [a if x == b else x for x in label]
    lin = module * PIX + col * ROWS + row
    groups = {}
    for i in range(n):
        groups.setdefault(label[i], []).append(i)
    ids = np.full(n, -1, dtype=np.int64)
    kept = []
    for members in groups.values():
        cid = int(min(lin[m] for m in members))
        ch = int(sum(int(adc[m]) for m in members)) & 0xFFFFFFFF
        if ch >= cut:
            kept.append((cid, ch, len(members)))
            for m in members:
                ids[m] = cid
    kept.sort()
    return ids, kept


def patterns_event(codes, R, C, r0, c0, rng):
    """Event with one binary R x C pattern per module (bit k <-> row k % R, col k // R),
    placed with its top-left corner at (r0, c0).  Returns (event dict, fired stack)."""
    codes = np.asarray(codes, dtype=np.int64)
    P = codes.size
    k = np.arange(R * C)
    fired_cm = ((codes[:, None] >> k[None, :]) & 1).astype(bool)      # (P, R*C) column-major
    fired = fired_cm.reshape(P, C, R).transpose(0, 2, 1)                # (P, R, C)
    p, r, c = np.nonzero(fired)
    ev = {
        "module": p.astype(np.uint16),
        "row": (r0 + r).astype(np.uint16),
        "col": (c0 + c).astype(np.uint16),
        "adc": rng.integers(0, 4001, p.size).astype(np.uint16),
        "n_modules": int(P),
    }
    return ev, fired


def expected_from_labels(ev, fired, lab, R, r0, c0, cut):
    """Expected per-digi ids and kept clusters for a ``patterns_event``."""
    p, r, c = np.nonzero(fired)
    L = lab[p, r, c].astype(np.int64)
    ids = p * PIX + (c0 + L // R) * ROWS + (r0 + L % R)
    adc = ev["adc"].astype(np.int64)
    uid, inv = np.unique(ids, return_inverse=True)
    charge = np.bincount(inv, weights=adc, minlength=uid.size).astype(np.int64)
    size = np.bincount(inv, minlength=uid.size).astype(np.int64)
    keep = charge >= cut
    digi = np.where(keep[inv], ids, -1)
    return digi, uid[keep], charge[keep], size[keep]
