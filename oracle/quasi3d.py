"""Plain float64 simulation of the quasi-3D variant: several cells per site.

Test infrastructure: part of the CPU oracle (see oracle/__init__.py).

The paper's own model is quasi-three-dimensional, a lattice site holding many
cells rather than one (Introduction, on the authors' earlier CA models;
Materials and Methods, where a small number of sites holds a much larger
number of cells).  It does not print how the cells of a site interact, so this
variant fixes the following rules on top of the 2D model of oracle/sim.py; with
C = 1 every rule below is the 2D model's.

  * Each site holds C cell slots; cells[z, y, x] is the word of slot z at site
    (y, x), in the 2D word format.  The fields stay two-dimensional.
  * The random words of slot z at site s (s = y L + x) are the Philox block of
    site counter z L^2 + s, so slot 0 draws what the 2D model draws.
  * Initial state: slot 0 is the 2D model's initial lattice, the other slots
    are EMPTY.
  * Irradiation: every live cell as in the 2D model (its class, and with the
    oxygen effect the oxygen bin of its site).
  * Activity of a site: the mean over its C slots of act[state], so a column of
    C identical cells acts like one 2D cell of that state.
  * Cell update of each cell as in the 2D model, with its site's fields and
    these division rules: the free places of a cell are the EMPTY slots of its
    own site and of its four von Neumann neighbours, taken in the order own
    site, N, E, S, W and within a site by slot; m counts them.  A ready cell
    proposes the k-th free place, k = floor(w0 m / 2^32), with the 64-bit key
    ((w2 >> 3) << 8) | (d << 5) | z: z its slot, d = 4 for its own site and
    otherwise its direction as seen from the target (N 0, E 1, S 2, W 3).  Each
    EMPTY slot with proposers takes the smallest key; daughter and winning
    parent get age 0.
  * The live count is the number of PROLIF and QUIESC cells over all slots.
"""
import numpy as np

from . import sim
from .model import AGE_MAX, DEAD, EMPTY, PROLIF, QUIESC, Params
from .philox import site_words
from .protocol import events, validate

OWN = 4
NONE_KEY64 = np.uint64(0xFFFFFFFFFFFFFFFF)
MAX_SLOTS = 32


def slot_draw(n, r, p, seed, L):
    """Draw function over flat slot indices z L^2 + s."""
    return lambda idx: site_words(np.asarray(idx, np.int64), n, r, p, seed)


def init_state(params: Params, L, C, p, r, seed):
    fields, plane = sim.init_state(params, L, p, r, seed)
    cells = np.zeros((C, L, L), np.int64)
    cells[0] = plane
    return fields, cells


def live_count(cells):
    st = np.asarray(cells, np.int64) & 3
    return int(np.count_nonzero((st == PROLIF) | (st == QUIESC)))


def irradiate(cells, thresholds, draw, params: Params, fields=None):
    """One fraction on every slot (each slot plane as a 2D lattice whose site
    counters are offset by z L^2)."""
    C, L, _ = cells.shape
    out = np.empty_like(cells)
    for z in range(C):
        out[z] = sim.irradiate(cells[z], thresholds, lambda s, z=z: draw(z * L * L + np.asarray(s)), params, fields)
    return out


def activity(cells, params: Params):
    """Mean over the slots of act[state]."""
    C = cells.shape[0]
    act = np.asarray(params.act, np.float64)[np.asarray(cells, np.int64) & 3]
    return act.sum(axis=0) / C


# site offsets of the groups own, N, E, S, W and the code d of a proposer of
# each group as seen from its target
GROUP_DY = (0, -1, 0, 1, 0)
GROUP_DX = (0, 0, 1, 0, -1)
GROUP_CODE = (OWN, 2, 3, 0, 1)


def cell_update(cells, fields, draw, params: Params):
    """Synchronous cell update of every slot from the snapshot `cells` [C, L, L]
    and the fields after diffusion; draw(flat slot indices) -> words [4, n]."""
    C, H, W = cells.shape
    cells = np.asarray(cells, np.int64)
    state, age = sim.unpack(cells)
    doom = sim.doomed(cells)
    O, G, Hf = (np.broadcast_to(f, (C, H, W)) for f in fields)
    new_state, new_age = state.copy(), age.copy()
    new_age[state == EMPTY] = 0
    older = np.minimum(age + 1, AGE_MAX)

    dead = state == DEAD
    new_age[dead] = older[dead]
    lysed = dead & (older >= params.T_lys)
    new_state[lysed] = EMPTY
    new_age[lysed] = 0

    live = (state == PROLIF) | (state == QUIESC)
    necrotic = live & ((G < params.th_Gd) | (O < params.th_Od) | (Hf > params.th_Hd))
    starving = live & ~necrotic & ((O < params.th_Oq) | (G < params.th_Gq))
    cycling = live & ~necrotic & ~starving
    new_state[necrotic] = DEAD
    new_age[necrotic] = 0
    new_state[starving] = QUIESC
    new_state[cycling] = PROLIF
    new_age[cycling] = older[cycling]
    new_doom = np.where(live & ~necrotic, doom, 0)

    empty = state == EMPTY
    nfree = empty.sum(axis=0)                                  # free slots per site
    padded = np.pad(nfree, 1)                                  # 0 outside the lattice
    group_free = np.stack([padded[1 + dy:1 + dy + H, 1 + dx:1 + dx + W] for dy, dx in zip(GROUP_DY, GROUP_DX)])
    m = group_free.sum(axis=0)                                 # [H, W]
    # slot indices of each site with its EMPTY slots first, in slot order
    free_order = np.argsort(~empty, axis=0, kind="stable")

    if params.mitotic_death:
        marked = cycling & (doom == 1) & (age >= params.T_min)
        zz, yy, xx = np.nonzero(marked)
        if len(zz):
            dies = draw((zz * H + yy) * W + xx)[3].astype(np.uint64) < np.uint64(params.T_div)
            new_state[zz[dies], yy[dies], xx[dies]] = DEAD
            new_age[zz[dies], yy[dies], xx[dies]] = 0
            new_doom[zz[dies], yy[dies], xx[dies]] = 0
        cycling = cycling & (doom == 0)
    cand = cycling & (age >= params.T_min) & (m[None] >= 1)
    zs, ys, xs = np.nonzero(cand)
    if len(zs):
        w = draw((zs * H + ys) * W + xs).astype(np.uint64)
        ready = w[3] < np.uint64(params.T_div)
        zs, ys, xs, w = zs[ready], ys[ready], xs[ready], w[:, ready]
    if len(zs):
        mm = m[ys, xs].astype(np.uint64)
        k = ((w[0] * mm) >> np.uint64(32)).astype(np.int64)
        counts = group_free[:, ys, xs]                          # [5, n]
        ends = np.cumsum(counts, axis=0)
        g = np.argmax(ends > k[None, :], axis=0)               # group of the k-th free place
        j = k - (ends[g, np.arange(len(k))] - counts[g, np.arange(len(k))])
        ty = ys + np.asarray(GROUP_DY)[g]
        tx = xs + np.asarray(GROUP_DX)[g]
        tz = free_order[j, ty, tx]
        assert np.all(empty[tz, ty, tx])
        code = np.asarray(GROUP_CODE, np.uint64)[g]
        key = ((w[2] >> np.uint64(3)) << np.uint64(8)) | (code << np.uint64(5)) | zs.astype(np.uint64)
        best = np.full((C, H, W), NONE_KEY64, dtype=np.uint64)
        np.minimum.at(best, (tz, ty, tx), key)
        won = best[tz, ty, tx] == key
        born = best != NONE_KEY64
        new_state[born] = PROLIF
        new_age[born] = 0
        new_doom[born] = 0
        new_age[zs[won], ys[won], xs[won]] = 0
    return sim.pack(new_state, new_age, new_doom)


def step(fields, cells, n, thresholds, p, r, seed, params: Params, substeps, thresholds_mid=None):
    """One step of one instance, in the 2D model's order (irradiation, frozen
    activity, FTCS sub-steps with a half-hour fraction between them, cell
    update)."""
    L = cells.shape[1]
    draw = slot_draw(n, r, p, seed, L)
    if thresholds is not None:
        cells = irradiate(cells, thresholds, draw, params, fields)
    act = activity(cells, params)
    first = substeps // 2 if thresholds_mid is not None else substeps
    for _ in range(first):
        fields = sim.diffuse_substep(fields, act, params)
    if thresholds_mid is not None:
        cells = irradiate(cells, thresholds_mid, slot_draw(sim.MID_STEP | n, r, p, seed, L), params, fields)
        act = activity(cells, params)
        for _ in range(substeps - first):
            fields = sim.diffuse_substep(fields, act, params)
    cells = cell_update(cells, fields, draw, params)
    return fields, cells


def run_instance(params: Params, L, C, nsteps, substeps, ev, p, r, seed, state=None, n0=0, half_hour=False):
    """Steps n0 .. n0+nsteps-1 from `state` (or the initial state); returns
    (fields, cells, live count after each step)."""
    fields, cells = init_state(params, L, C, p, r, seed) if state is None else state
    evmap = {(t if half_hour else 2 * t): thr for t, thr in ev}
    traj = np.zeros(nsteps, np.int64)
    for i in range(nsteps):
        n = n0 + i
        fields, cells = step(fields, cells, n, evmap.get(2 * n), p, r, seed, params, substeps,
                             thresholds_mid=evmap.get(2 * n + 1))
        traj[i] = live_count(cells)
    return fields, cells, traj


def simulate(params: Params, L, C, horizon, substeps, R, seed, dose, gap, nfrac, K, cap, half_hour=False):
    """live[p, r] after `horizon` steps (-1 for invalid protocols) and
    fitness[p] = mean over replicas."""
    dose = np.asarray(dose, np.float32).reshape(-1, K)
    gap = np.asarray(gap, np.int64).reshape(-1, K)
    nfrac = np.asarray(nfrac).reshape(-1)
    P = len(nfrac)
    status = validate(dose, gap, nfrac, K, cap)
    live = np.full((P, R), -1, np.int64)
    fitness = np.full(P, np.nan)
    for p in range(P):
        if status[p]:
            continue
        ev = events(dose[p], gap[p], nfrac[p], horizon, params, half_hour)
        for r in range(R):
            if horizon == 0:
                live[p, r] = live_count(init_state(params, L, C, p, r, seed)[1])
            else:
                live[p, r] = run_instance(params, L, C, horizon, substeps, ev, p, r, seed, half_hour=half_hour)[2][-1]
        fitness[p] = live[p].mean()
    return live, fitness
