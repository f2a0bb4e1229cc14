"""Plain float64 simulation of the tumour / irradiation lattice automaton.

Test infrastructure: part of the CPU oracle (see oracle/__init__.py).

What the paper fixes about the simulated method (Materials and Methods): a
cellular automaton of spheroid cells on a lattice, coupled to diffusing
nutrient (oxygen, glucose) and waste (acidity) fields; cells cycle, turn
quiescent or die according to local conditions, divide into free neighbouring
sites, and respond to each radiotherapy fraction; the fitness of a protocol is
read from the number of occupied sites at the end ("The fitness function",
equation final_fit_fun), averaged over replicate simulations.  The equations
are not printed in the paper; the synthetic model below fixes them:

Per instance (protocol p, replica r) and step n = 0 .. N-1 (one model hour):
  1. irradiation, if a fraction falls on step n: each live cell of sensitivity
     class c survives iff w1 < T_c (linear-quadratic threshold), else it is
     DEAD with age 0; with the oxygen effect the threshold also depends on
     the oxygen bin of the site's current O (protocol.oxygen_thresholds);
  2. the activity map a = act[state] is frozen until the next fraction or the
     end of the hour;
  3. `substeps` explicit FTCS updates of the three fields,
     c' = c + lam (c_N + c_S + c_E + c_W - 4 c) - kappa a   (O, G; then max(.,0))
     H' = H + lam (H_N + H_S + H_E + H_W - 4 H) + kappa a,
     with Dirichlet ghost values outside the lattice; a fraction at the half
     hour (protocols timed in 30-minute units) is applied as in 1 after
     substeps // 2 of them, with w1 from the block of step word n | 2^31, and
     the activity map is rebuilt from the surviving cells;
  4. a synchronous cell update from the snapshot taken after the irradiation
     and the fields after step 3 (see cell_update);
  5. the live count (PROLIF + QUIESC) is recorded.

Cell words: bits 0-1 state (EMPTY, PROLIF, QUIESC, DEAD), bits 2-9 age in
hours (saturating at 255), bit 14 the mark of a lethally hit cell awaiting
mitotic death (params.mitotic_death).
"""
import numpy as np

from .model import AGE_MAX, DEAD, DOOM, EMPTY, PROLIF, QUIESC, Params
from .philox import INIT_STEP, site_words
from .protocol import events, oxygen_bin, validate

# Von Neumann neighbours in the fixed order N, E, S, W (row y grows southwards).
DY = (-1, 0, 1, 0)
DX = (0, 1, 0, -1)
NONE_KEY = 0xFFFFFFFF


def pack(state, age, doom=0):
    return (np.asarray(state, np.int64) & 3) | (np.asarray(age, np.int64) << 2) | (np.asarray(doom, np.int64) * DOOM)


def doomed(cells):
    """1 where a lethally hit cell awaits mitotic death (bit 14 of the word)."""
    return (np.asarray(cells, np.int64) >> 14) & 1


def unpack(cells):
    cells = np.asarray(cells, np.int64)
    return cells & 3, (cells >> 2) & 0xFF


def live_count(cells):
    state, _ = unpack(cells)
    return int(np.count_nonzero((state == PROLIF) | (state == QUIESC)))


def init_state(params: Params, L, p, r, seed):
    """Initial state: uniform fields; a disc of PROLIF cells at the centre.

    Sites with (x - c)^2 + (y - c)^2 <= radius^2, c = L // 2, hold PROLIF cells
    whose age is floor(w0 * A0 / 2**32), w0 from the block at step 0xFFFFFFFF.
    """
    fields = np.empty((3, L, L), dtype=np.float64)
    for f in range(3):
        fields[f] = params.init[f]
    yy, xx = np.mgrid[0:L, 0:L]
    c = L // 2
    disc = (xx - c) ** 2 + (yy - c) ** 2 <= params.seed_radius ** 2
    ys, xs = np.nonzero(disc)
    w0 = site_words(ys * L + xs, INIT_STEP, r, p, seed)[0].astype(np.uint64)
    age = ((w0 * np.uint64(params.A0)) >> np.uint64(32)).astype(np.int64)
    cells = np.zeros((L, L), dtype=np.int64)
    cells[ys, xs] = pack(PROLIF, age)
    return fields, cells


def sensitivity_class(state, age, params: Params):
    """0/1/2 for proliferating cells by age band, 3 for quiescent cells."""
    a0, a1 = params.class_age
    cls = np.where(age < a0, 0, np.where(age < a1, 1, 2))
    return np.where(state == QUIESC, 3, cls)


def irradiate(cells, thresholds, draw, params: Params, fields=None):
    """Apply one fraction: a live cell survives iff its word w1 < T[class]
    (with the oxygen effect, T[class][oxygen bin of the site's O])."""
    H, W = cells.shape
    state, age = unpack(cells)
    live = (state == PROLIF) | (state == QUIESC)
    ys, xs = np.nonzero(live)
    if len(ys) == 0:
        return cells.copy()
    w1 = draw(ys * W + xs)[1].astype(np.int64)
    cls = sensitivity_class(state[ys, xs], age[ys, xs], params)
    if params.oxygen_effect:
        bins = np.array([oxygen_bin(fields[0, y, x], params) for y, x in zip(ys, xs)], dtype=np.int64)
        thr = np.asarray(thresholds, dtype=np.int64)[cls, bins]
    else:
        thr = np.asarray(thresholds, dtype=np.int64)[cls]
    killed = w1 >= thr
    out = cells.copy()
    if params.mitotic_death:        # the cell lives on, marked, until it next divides
        out[ys[killed], xs[killed]] |= DOOM
    else:
        out[ys[killed], xs[killed]] = pack(DEAD, 0)
    return out


def activity(cells, params: Params):
    state, _ = unpack(cells)
    return np.asarray(params.act, dtype=np.float64)[state]


def diffuse_substep(fields, act, params: Params):
    """One explicit FTCS update of (O, G, H) with Dirichlet ghost values."""
    out = np.empty_like(fields)
    for f in range(3):
        c = fields[f]
        pad = np.pad(c, 1, mode="constant", constant_values=params.ghost[f])
        nb = pad[:-2, 1:-1] + pad[2:, 1:-1] + pad[1:-1, 2:] + pad[1:-1, :-2]
        new = c + params.lam[f] * (nb - 4.0 * c)
        if f < 2:
            new = np.maximum(new - params.kappa[f] * act, 0.0)
        else:
            new = new + params.kappa[f] * act
        out[f] = new
    return out


def free_neighbours(empty):
    """free[d, y, x]: the neighbour of (y, x) in direction d is an EMPTY site."""
    H, W = empty.shape
    free = np.zeros((4, H, W), dtype=bool)
    free[0, 1:, :] = empty[:-1, :]
    free[1, :, :-1] = empty[:, 1:]
    free[2, :-1, :] = empty[1:, :]
    free[3, :, 1:] = empty[:, :-1]
    return free


def cell_update(cells, fields, draw, params: Params):
    """Synchronous cell update of one step.

    From the snapshot `cells` and the fields after diffusion:
      EMPTY: stays EMPTY (word 0) unless it receives a daughter.
      DEAD: age + 1; once age >= T_lys the site becomes EMPTY (free next step).
      live: DEAD (age 0) if G < th_Gd or O < th_Od or H > th_Hd; else QUIESC if
        O < th_Oq or G < th_Gq (age kept); else PROLIF.
      PROLIF with age >= T_min and m >= 1 EMPTY von Neumann neighbours draws a
        block; it is ready iff w3 < T_div and then proposes the k-th free
        neighbour in N, E, S, W order, k = floor(w0 m / 2**32), with key
        ((w2 >> 3) << 2) | d, d its own direction as seen from the target.
      Every EMPTY site with proposers takes the smallest key: the daughter there
        and the winning parent both get age 0.  Every other PROLIF cell ages by 1.
      With mitotic death, a marked (lethally hit) PROLIF cell with age >= T_min
        draws its block whatever its neighbours; when ready (w3 < T_div) it
        dies (DEAD, age 0) instead of dividing.  Live cells keep the mark;
        dead ones drop it.
    """
    H, W = cells.shape
    state, age = unpack(cells)
    doom = doomed(cells)
    O, G, Hf = fields
    new_state, new_age = state.copy(), age.copy()
    new_age[state == EMPTY] = 0        # an EMPTY site's word is always 0
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
    free = free_neighbours(state == EMPTY)
    m = free.sum(axis=0)
    if params.mitotic_death:
        marked = cycling & (doom == 1) & (age >= params.T_min)
        my, mx = np.nonzero(marked)
        if len(my):
            dies = draw(my * W + mx)[3].astype(np.uint64) < np.uint64(params.T_div)
            new_state[my[dies], mx[dies]] = DEAD
            new_age[my[dies], mx[dies]] = 0
            new_doom[my[dies], mx[dies]] = 0
        cycling = cycling & (doom == 0)
    cand = cycling & (age >= params.T_min) & (m >= 1)
    ys, xs = np.nonzero(cand)
    if len(ys):
        w = draw(ys * W + xs).astype(np.uint64)
        ready = w[3] < np.uint64(params.T_div)
        ys, xs, w = ys[ready], xs[ready], w[:, ready]
    if len(ys):
        mm = m[ys, xs].astype(np.uint64)
        k = ((w[0] * mm) >> np.uint64(32)).astype(np.int64)
        # direction of the k-th free neighbour (0-based) in N, E, S, W order
        fr = free[:, ys, xs]                       # (4, n)
        rank = np.cumsum(fr, axis=0) - 1           # rank among free ones
        dirn = np.argmax(fr & (rank == k[None, :]), axis=0)
        ty = ys + np.asarray(DY)[dirn]
        tx = xs + np.asarray(DX)[dirn]
        key = ((w[2] >> np.uint64(3)) << np.uint64(2)) | ((dirn + 2) % 4).astype(np.uint64)
        best = np.full((H, W), NONE_KEY, dtype=np.uint64)
        np.minimum.at(best, (ty, tx), key)
        won = best[ty, tx] == key
        born = best != NONE_KEY
        new_state[born] = PROLIF
        new_age[born] = 0
        new_age[ys[won], xs[won]] = 0
    return pack(new_state, new_age, new_doom)


MID_STEP = 0x80000000   # step word bit of the draws of a fraction at the half hour


def step(fields, cells, n, thresholds, p, r, seed, params: Params, substeps, thresholds_mid=None):
    """Advance one instance by one step; `thresholds` (start of the hour) and
    `thresholds_mid` (its middle) are None without a fraction."""
    draw = lambda sites: site_words(sites, n, r, p, seed)
    if thresholds is not None:
        cells = irradiate(cells, thresholds, draw, params, fields)
    act = activity(cells, params)
    first = substeps // 2 if thresholds_mid is not None else substeps
    for _ in range(first):
        fields = diffuse_substep(fields, act, params)
    if thresholds_mid is not None:
        cells = irradiate(cells, thresholds_mid, lambda sites: site_words(sites, MID_STEP | n, r, p, seed), params,
                          fields)
        act = activity(cells, params)
        for _ in range(substeps - first):
            fields = diffuse_substep(fields, act, params)
    cells = cell_update(cells, fields, draw, params)
    return fields, cells


def run_instance(params: Params, L, nsteps, substeps, ev, p, r, seed, state=None, n0=0, half_hour=False):
    """Run steps n0 .. n0+nsteps-1; returns (fields, cells, live count per step).
    `ev` holds (time, thresholds) with times in steps, or in half-hours when
    half_hour is set."""
    if state is None:
        fields, cells = init_state(params, L, p, r, seed)
    else:
        fields, cells = state
    evmap = {(t if half_hour else 2 * t): thr for t, thr in ev}
    traj = np.zeros(nsteps, dtype=np.int64)
    for i in range(nsteps):
        n = n0 + i
        fields, cells = step(fields, cells, n, evmap.get(2 * n), p, r, seed, params, substeps,
                             thresholds_mid=evmap.get(2 * n + 1))
        traj[i] = live_count(cells)
    return fields, cells, traj


def simulate(params: Params, L, horizon, substeps, R, seed, dose, gap, nfrac, K, cap, half_hour=False):
    """Whole batch: live[p, r] after `horizon` steps and fitness[p] = mean_r live
    (delays in half-hours with half_hour=True).

    Invalid protocols get live = -1 and fitness NaN.  The paper's own score is
    L*L - fitness (the maximal number of occupiable sites minus the mean count).
    """
    dose = np.asarray(dose, np.float32).reshape(-1, K)
    gap = np.asarray(gap, np.int64).reshape(-1, K)
    nfrac = np.asarray(nfrac).reshape(-1)
    P = len(nfrac)
    status = validate(dose, gap, nfrac, K, cap)
    live = np.full((P, R), -1, dtype=np.int64)
    fitness = np.full(P, np.nan)
    for p in range(P):
        if status[p]:
            continue
        ev = events(dose[p], gap[p], nfrac[p], horizon, params, half_hour)
        for r in range(R):
            live[p, r] = run_instance(params, L, horizon, substeps, ev, p, r, seed, half_hour=half_hour)[2][-1]
        fitness[p] = live[p].mean()
    return live, fitness
