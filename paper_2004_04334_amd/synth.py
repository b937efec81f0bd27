"""Seeded synthetic pixel-detector events (the workloads of the five configurations).

This module only *draws inputs*: fired pixels ("digis") as a structure of arrays
``module, row, col, adc`` (all ``uint16``), grouped by ascending module id and
shuffled within each module.  It contains none of the clustering arithmetic and
is shared by the CPU oracle tests and the device tests alike.

Geometry: a module is 160 rows x 416 columns.  Events stand in for real detector
data, which the paper does not ship (its example producers only name the
"raw -> clusters -> hits" chain, Figure 1 / Sec. 3); the recipe is:

* RNG: ``PCG64(SeedSequence(entropy=2004_04334, spawn_key=(config_id, event_idx)))``.
* ADC: integers uniform in [100, 4000].
* Cluster sizes: geometric on {1,2,...} (p=0.25, mean 4; p=0.025, mean 40 for hot
  modules).  A cluster grows from a uniform seed; each new pixel is a +-1 step from
  a uniformly chosen member, along the row axis with probability 0.75 (so clusters
  are elongated along columns), else along the column axis, clipped to the module;
  an already-fired target is redrawn.  Touching clusters are allowed to merge.
* Noise: uniform pixels whose 3x3 neighbourhood is empty when placed.
* Cluster:noise pixel ratio 10:1.
"""
from __future__ import annotations

import numpy as np

ROWS = 160
COLS = 416
PIXELS = ROWS * COLS
N_MODULES_FULL = 1856
ENTROPY = 2004_04334

# configuration ids used in the seed's spawn key
CFG_PLAIN, CFG_ASYNC, CFG_BATCH, CFG_SERVE, CFG_STRESS, CFG_TEST = 0, 1, 2, 3, 4, 9
CFG_STRESS_ALL = 5   # the stress configuration with 10 % of all modules hot


def rng_for(config_id: int, event_idx: int) -> np.random.Generator:
    ss = np.random.SeedSequence(entropy=ENTROPY, spawn_key=(int(config_id), int(event_idx)))
    return np.random.Generator(np.random.PCG64(ss))


class _Canvas:
    """Occupancy of the active modules of one event (dense index per module)."""

    def __init__(self, n_active: int):
        # one pixel of padding on every side makes neighbourhood tests branch-free
        self.fired = np.zeros((n_active, ROWS + 2, COLS + 2), dtype=bool)

    def is_fired(self, m, r, c):
        return self.fired[m, r + 1, c + 1]

    def set(self, m, r, c):
        self.fired[m, r + 1, c + 1] = True

    def neighbourhood_empty(self, m, r, c):
        f = self.fired
        ok = np.ones(np.shape(m), dtype=bool)
        for dr in (0, 1, 2):
            for dc in (0, 1, 2):
                ok &= ~f[m, r + dr, c + dc]
        return ok


def _unique_first(keys: np.ndarray) -> np.ndarray:
    """Indices of the first occurrence of each distinct key."""
    _, first = np.unique(keys, return_index=True)
    return np.sort(first)


def _grow_clusters(rng, canvas, cl_mod, sizes, p_row=0.75):
    """Grow clusters (all at once, one pixel per cluster per round).

    Returns (m, r, c) of every pixel placed; a cluster whose growth keeps
    failing stops early (the caller tops the pixel count up).
    """
    C = len(sizes)
    if C == 0:
        e = np.zeros(0, dtype=np.int64)
        return e, e, e
    maxs = int(sizes.max())
    R = np.zeros((C, maxs), dtype=np.int32)
    K = np.zeros((C, maxs), dtype=np.int32)
    # seeds: uniform, unfired, distinct
    need = np.arange(C)
    while need.size:
        sr = rng.integers(0, ROWS, need.size)
        sc = rng.integers(0, COLS, need.size)
        m = cl_mod[need]
        free = ~canvas.is_fired(m, sr, sc)
        cand = np.nonzero(free)[0]
        if cand.size:
            keys = (m[cand].astype(np.int64) * ROWS + sr[cand]) * COLS + sc[cand]
            acc = cand[_unique_first(keys)]
            canvas.set(m[acc], sr[acc], sc[acc])
            R[need[acc], 0] = sr[acc]
            K[need[acc], 0] = sc[acc]
            keep = np.ones(need.size, dtype=bool)
            keep[acc] = False
            need = need[keep]
    k = np.ones(C, dtype=np.int64)
    tries = np.zeros(C, dtype=np.int64)
    limit = 16 * sizes + 16
    active = np.nonzero(k < sizes)[0]
    while active.size:
        u = (rng.random(active.size) * k[active]).astype(np.int64)
        mr = R[active, u]
        mc = K[active, u]
        along_row = rng.random(active.size) < p_row
        sign = rng.integers(0, 2, active.size) * 2 - 1
        nr = np.clip(mr + np.where(along_row, sign, 0), 0, ROWS - 1)
        nc = np.clip(mc + np.where(along_row, 0, sign), 0, COLS - 1)
        m = cl_mod[active]
        free = ~canvas.is_fired(m, nr, nc)
        cand = np.nonzero(free)[0]
        acc = np.zeros(0, dtype=np.int64)
        if cand.size:
            keys = (m[cand].astype(np.int64) * ROWS + nr[cand]) * COLS + nc[cand]
            acc = cand[_unique_first(keys)]
            ci = active[acc]
            canvas.set(m[acc], nr[acc], nc[acc])
            R[ci, k[ci]] = nr[acc]
            K[ci, k[ci]] = nc[acc]
            k[ci] += 1
        failed = np.ones(active.size, dtype=bool)
        failed[acc] = False
        tries[active[failed]] += 1
        active = active[(k[active] < sizes[active]) & (tries[active] < limit[active])]
    mask = np.arange(maxs)[None, :] < k[:, None]
    mm = np.broadcast_to(cl_mod[:, None], (C, maxs))[mask]
    return mm.astype(np.int64), R[mask].astype(np.int64), K[mask].astype(np.int64)


def _place_noise(rng, canvas, mod_idx, count):
    """Place ``count`` isolated pixels in module ``mod_idx`` (sequential acceptance)."""
    out_r, out_c = [], []
    guard = 0
    while len(out_r) < count and guard < 10_000:
        guard += 1
        want = count - len(out_r)
        rr = rng.integers(0, ROWS, 4 * want + 8)
        cc = rng.integers(0, COLS, 4 * want + 8)
        mm = np.full(rr.size, mod_idx)
        ok = canvas.neighbourhood_empty(mm, rr, cc)
        for r, c in zip(rr[ok].tolist(), cc[ok].tolist()):
            if len(out_r) >= count:
                break
            if canvas.neighbourhood_empty(mod_idx, r, c):
                canvas.set(mod_idx, r, c)
                out_r.append(r)
                out_c.append(c)
    return np.asarray(out_r, dtype=np.int64), np.asarray(out_c, dtype=np.int64)


def _fill_modules(rng, mods, cluster_px, noise_px, p_geom):
    """Fill each listed module with the requested cluster and noise pixel counts.

    ``mods`` are module ids (ascending); returns (module, row, col) arrays.
    """
    n_act = len(mods)
    canvas = _Canvas(n_act)
    cluster_px = np.asarray(cluster_px, dtype=np.int64)
    noise_px = np.asarray(noise_px, dtype=np.int64)
    placed = np.zeros(n_act, dtype=np.int64)
    pieces = []
    # clusters, topped up until every module holds exactly its cluster pixel count
    for _round in range(64):
        deficit = cluster_px - placed
        if not (deficit > 0).any():
            break
        cl_mod, sizes = [], []
        for i in np.nonzero(deficit > 0)[0]:
            d = int(deficit[i])
            s = rng.geometric(p_geom, size=max(4, int(2 * d * p_geom) + 4))
            cs = np.cumsum(s)
            j = int(np.searchsorted(cs, d))
            if j >= s.size:           # extremely unlikely; take what we have
                j = s.size - 1
            s = s[: j + 1].copy()
            s[-1] -= int(cs[j]) - d if cs[j] > d else 0
            cl_mod.append(np.full(s.size, i, dtype=np.int64))
            sizes.append(s.astype(np.int64))
        cl_mod = np.concatenate(cl_mod)
        sizes = np.concatenate(sizes)
        m, r, c = _grow_clusters(rng, canvas, cl_mod, sizes)
        pieces.append((m, r, c))
        placed += np.bincount(m, minlength=n_act)
    for i in range(n_act):
        if noise_px[i] > 0:
            r, c = _place_noise(rng, canvas, i, int(noise_px[i]))
            pieces.append((np.full(r.size, i, dtype=np.int64), r, c))
    m = np.concatenate([p[0] for p in pieces]) if pieces else np.zeros(0, np.int64)
    r = np.concatenate([p[1] for p in pieces]) if pieces else np.zeros(0, np.int64)
    c = np.concatenate([p[2] for p in pieces]) if pieces else np.zeros(0, np.int64)
    return np.asarray(mods, dtype=np.int64)[m], r, c


def _finish(rng, m, r, c, n_modules, extra=None):
    """Group by ascending module, shuffle within modules, draw ADC."""
    if extra is not None:
        m = np.concatenate([m, extra[0]])
        r = np.concatenate([r, extra[1]])
        c = np.concatenate([c, extra[2]])
    perm = rng.permutation(m.size)
    order = perm[np.argsort(m[perm], kind="stable")]
    m, r, c = m[order], r[order], c[order]
    adc = rng.integers(100, 4001, m.size)
    return {
        "module": m.astype(np.uint16),
        "row": r.astype(np.uint16),
        "col": c.astype(np.uint16),
        "adc": adc.astype(np.uint16),
        "n_modules": int(n_modules),
    }


def _split_10_to_1(total):
    total = np.asarray(total, dtype=np.int64)
    noise = np.rint(total / 11.0).astype(np.int64)
    return total - noise, noise


def plain_event(event_idx: int, n_modules: int = 64):
    """Configuration 1: 64 modules, 666 cluster + 67 noise pixels each (46,912 digis)."""
    rng = rng_for(CFG_PLAIN, event_idx)
    mods = np.arange(n_modules)
    m, r, c = _fill_modules(rng, mods, np.full(n_modules, 666), np.full(n_modules, 67), 0.25)
    return _finish(rng, m, r, c, n_modules)


def async_event(event_idx: int, n_modules: int = N_MODULES_FULL):
    """Configuration 2: 1,856 modules, Poisson(24.5) cluster + Poisson(2.45) noise pixels
    per module (about 50k digis)."""
    rng = rng_for(CFG_ASYNC, event_idx)
    cl = rng.poisson(24.5, n_modules)
    nz = rng.poisson(2.45, n_modules)
    mods = np.nonzero(cl + nz)[0]
    m, r, c = _fill_modules(rng, mods, cl[mods], nz[mods], 0.25)
    return _finish(rng, m, r, c, n_modules)


def _lognormal_modules(rng, n_target, n_modules, exclude=()):
    """Draw modules without replacement with log-normal occupancy (median 0.5 %,
    sigma 0.92, clipped to [0.05 %, 5 %]) until ``n_target`` pixels are reached."""
    pool = np.setdiff1d(rng.permutation(n_modules), np.asarray(exclude, dtype=np.int64),
                        assume_unique=False)
    pool = rng.permutation(pool)
    occ = np.clip(rng.lognormal(np.log(0.005), 0.92, pool.size), 0.0005, 0.05)
    px = np.maximum(1, np.rint(occ * PIXELS).astype(np.int64))
    cs = np.cumsum(px)
    j = int(np.searchsorted(cs, n_target))
    if j >= pool.size:
        raise ValueError("event larger than the module pool allows")
    px = px[: j + 1].copy()
    px[-1] -= int(cs[j]) - n_target
    if px[-1] == 0:
        px = px[:-1]
    mods = pool[: px.size]
    order = np.argsort(mods)
    return mods[order], px[order]


def batch_event(event_idx: int, n_modules: int = N_MODULES_FULL, lo=10_000, hi=120_000,
                config_id=CFG_BATCH):
    """Configuration 3 (and 4 with ``hi=200_000``): event size uniform in [lo, hi]."""
    rng = rng_for(config_id, event_idx)
    n_target = int(rng.integers(lo, hi + 1))
    mods, px = _lognormal_modules(rng, n_target, n_modules)
    cl, nz = _split_10_to_1(px)
    m, r, c = _fill_modules(rng, mods, cl, nz, 0.25)
    return _finish(rng, m, r, c, n_modules)


def serve_event(event_idx: int, n_modules: int = N_MODULES_FULL):
    """Configuration 4: event sizes uniform in [10k, 200k], module law of configuration 3."""
    return batch_event(event_idx, n_modules, 10_000, 200_000, config_id=CFG_SERVE)


def column_track(col: int):
    """A full-column, one-pixel-wide track: every row of one column."""
    r = np.arange(ROWS, dtype=np.int64)
    return r, np.full(ROWS, col, dtype=np.int64)


def serpentine(row_wise: bool):
    """One serpentine cluster filling every other line of a module, with the
    lines joined at alternating ends (row-wise: 33,359 pixels; column-wise: 33,487)."""
    rr, cc = [], []
    if row_wise:
        for k, row in enumerate(range(0, ROWS, 2)):
            rr.append(np.full(COLS, row)); cc.append(np.arange(COLS))
            if row + 2 < ROWS:
                rr.append(np.array([row + 1])); cc.append(np.array([COLS - 1 if k % 2 == 0 else 0]))
    else:
        for k, col in enumerate(range(0, COLS, 2)):
            rr.append(np.arange(ROWS)); cc.append(np.full(ROWS, col))
            if col + 2 < COLS:
                rr.append(np.array([ROWS - 1 if k % 2 == 0 else 0])); cc.append(np.array([col + 1]))
    return np.concatenate(rr).astype(np.int64), np.concatenate(cc).astype(np.int64)


def stress_event(event_idx: int, n_modules: int = N_MODULES_FULL, n_hot: int = 16, config: int = CFG_STRESS):
    """Configuration 5: 160 active modules = 16 hot modules at 20 % occupancy with
    mean-40 clusters + 142 modules of the configuration-3 law + a module holding only
    a full-column track + a module holding only a serpentine (row-wise on even
    events, column-wise on odd ones); about 310-330k digis.  With n_hot hot modules
    instead of 16 (stress_all_event) the rest is drawn the same way."""
    rng = rng_for(config, event_idx)
    chosen = rng.choice(n_modules, size=n_hot + 2, replace=False)
    hot, adv = np.sort(chosen[:n_hot]), chosen[n_hot:]
    hot_px = int(round(0.20 * PIXELS))
    hcl, hnz = _split_10_to_1(np.full(n_hot, hot_px))
    m1, r1, c1 = _fill_modules(rng, hot, hcl, hnz, 0.025)
    # 142 modules of the log-normal law (total drawn module by module)
    pool = np.setdiff1d(np.arange(n_modules), chosen)
    mods = np.sort(rng.choice(pool, size=142, replace=False))
    occ = np.clip(rng.lognormal(np.log(0.005), 0.92, 142), 0.0005, 0.05)
    px = np.maximum(1, np.rint(occ * PIXELS).astype(np.int64))
    cl, nz = _split_10_to_1(px)
    m2, r2, c2 = _fill_modules(rng, mods, cl, nz, 0.25)
    tr, tc = column_track(int(rng.integers(0, COLS)))
    sr, sc = serpentine(row_wise=(event_idx % 2 == 0))
    m3 = np.concatenate([np.full(tr.size, adv[0]), np.full(sr.size, adv[1])]).astype(np.int64)
    r3 = np.concatenate([tr, sr])
    c3 = np.concatenate([tc, sc])
    m = np.concatenate([m1, m2])
    r = np.concatenate([r1, r2])
    c = np.concatenate([c1, c2])
    return _finish(rng, m, r, c, n_modules, extra=(m3, r3, c3))


def stress_all_event(event_idx: int, n_modules: int = N_MODULES_FULL):
    """The stress configuration read literally: 10 % of all modules (186 of 1,856) hot
    at 20 % occupancy, plus the 142 sparse modules, the track and the serpentine; about
    2.5 million digis (a maximum-size case)."""
    return stress_event(event_idx, n_modules, n_hot=int(round(0.10 * n_modules)), config=CFG_STRESS_ALL)


def from_pixels(module, row, col, adc=None, n_modules=None, seed=0, shuffle=True):
    """Build an event from explicit pixels (tests): grouped by module, optionally
    shuffled within modules, ADC drawn if not given."""
    rng = rng_for(CFG_TEST, seed)
    module = np.asarray(module, dtype=np.int64)
    row = np.asarray(row, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    if adc is None:
        adc = rng.integers(100, 4001, module.size)
    adc = np.asarray(adc, dtype=np.int64)
    perm = rng.permutation(module.size) if shuffle else np.arange(module.size)
    order = perm[np.argsort(module[perm], kind="stable")]
    if n_modules is None:
        n_modules = int(module.max()) + 1 if module.size else 1
    return {
        "module": module[order].astype(np.uint16),
        "row": row[order].astype(np.uint16),
        "col": col[order].astype(np.uint16),
        "adc": adc[order].astype(np.uint16),
        "n_modules": int(n_modules),
    }


def n_digis(ev) -> int:
    return int(ev["module"].size)
