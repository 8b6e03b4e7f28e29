"""Seeded synthetic grids for the power-flow workloads.

Recipe (every draw comes from ``numpy.random.default_rng(seed)``):

Single-phase meshed transmission grid (stands in for the IEEE-30 replicas of
Sec. IV):
  * topology: random recursive tree (bus k attaches to a uniform j < k) plus
    ``n_extra`` uniform random chords between non-adjacent bus pairs;
  * branches: r ~ U[0.01, 0.05], x ~ U[0.05, 0.2], total line charging
    b ~ U[0, 0.04] pu, split b/2 to ground at each end (pi model);
  * bus 0 is the slack at 1.0 pu, angle 0; ``n_pv`` PV buses chosen uniformly
    with |V| = 1.02 and P ~ U[0.2, 0.8]; all others are PQ loads with
    P ~ U[0.05, 0.3] at power factor 0.9 lagging (Q = 0.4843 P);
  * ``balanced=True`` dispatches every PV bus at 0.6 x its draw and scales the
    loads so that total load equals total PV dispatch (the slack then covers
    the losses only).

Three-phase unbalanced radial feeder (stands in for the IEEE 906 LV feeder
replicas of Sec. IV):
  * topology: random recursive tree; bus 0 is the three-phase source at
    1.0 pu with phase angles 0, -120, +120 degrees;
  * laterals: about 20 % of the buses carry one or two phases; a lateral
    starts at a bus whose parent is three-phase (random 1- or 2-phase subset)
    and its whole subtree inherits that phase set;
  * branch impedance per km: z_s ~ U[0.3, 0.6] + jU[0.6, 1.2] ohm/km and a
    coupling k ~ U[0.3, 0.5]; Z = len * z_s * ((1-k) I + k 1 1^T), with
    len ~ U[0.05, 0.5] km; the sub-matrix of the present phases is used;
    per-unit on 12.47 kV line-to-line, Z_base = 155.5 ohm (per-phase power
    base 1/3 MVA);
  * loads: per bus, ZIP fractions ~ Dirichlet(1, 1, 1); per present phase
    P = s * U[0.5, 1.5] kW * U[0.7, 1.3] (the +-30 % imbalance), pf 0.9.

Replication-scale cases (Sec. IV's construction, at its sizes): copies of a
30-bus block joined by random links repeating base branches (48,000 buses),
and copies of a 906-bus feeder behind one substation branch (0.9K to 230K
buses); see ``replicate_polar`` and ``replicate_feeder``.

Batched scenarios: n ~ log-uniform[100, 5000], each with its own topology
drawn as for the 10,000-bus grid (0.3 n chords, 10 % PV, balanced), loads
perturbed per bus by a factor U[0.8, 1.2] applied to P and Q together.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

BASE_SEED = 20171128

PQ, PV, SLACK = 1, 2, 3

PF_LAG_TAN = math.tan(math.acos(0.9))

FEEDER_KV_LL = 12.47
FEEDER_S_BASE_MVA = 1.0
FEEDER_Z_BASE = FEEDER_KV_LL ** 2 / FEEDER_S_BASE_MVA  # ohm
FEEDER_S_PHASE_KVA = 1000.0 * FEEDER_S_BASE_MVA / 3.0
# Load scale of the 2,000-bus feeder workload.  Chosen once so that the
# lowest phase voltage of the seeded 2,000-bus feeder lies in [0.93, 0.96] pu.
FEEDER_LOAD_SCALE = 4.5


@dataclasses.dataclass
class PolarCase:
    """Single-phase grid: branch list, Ybus CSR and bus set-points."""

    name: str
    n: int
    f: np.ndarray          # int32 [m] from-bus
    t: np.ndarray          # int32 [m] to-bus
    r: np.ndarray          # float64 [m]
    x: np.ndarray          # float64 [m]
    b: np.ndarray          # float64 [m] total line charging
    row_ptr: np.ndarray    # int32 [n+1]
    col: np.ndarray        # int32 [nnz], sorted per row, diagonal present
    y: np.ndarray          # complex128 [nnz]
    bus_type: np.ndarray   # int8 [n]
    p_sp: np.ndarray       # float64 [n] specified injection (gen - load)
    q_sp: np.ndarray       # float64 [n]
    v_mag: np.ndarray      # float64 [n] |V| set-point (PV, slack); 1 for PQ
    v_ang: np.ndarray      # float64 [n] angle set-point (slack); 0 otherwise
    seed: int = 0

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def m(self) -> int:
        return int(self.f.shape[0])

    def with_injections(self, p_sp, q_sp, name=None) -> "PolarCase":
        return dataclasses.replace(self, p_sp=np.ascontiguousarray(p_sp, np.float64),
                                   q_sp=np.ascontiguousarray(q_sp, np.float64),
                                   name=name or self.name)


@dataclasses.dataclass
class CimCase:
    """Three-phase feeder over its present phase-nodes."""

    name: str
    n_bus: int
    n: int                 # phase-nodes
    node_bus: np.ndarray   # int32 [n]
    node_phase: np.ndarray # int32 [n] 0=a 1=b 2=c
    f: np.ndarray          # int32 [m] parent bus
    t: np.ndarray          # int32 [m] child bus
    zbr: np.ndarray        # complex128 [m,3,3] full per-unit branch impedance
    bus_phases: np.ndarray # int8 [n_bus,3] phase present
    row_ptr: np.ndarray
    col: np.ndarray
    y: np.ndarray
    node_type: np.ndarray  # int8 [n]: SLACK for source phase-nodes, PV for
                           # voltage-controlled generation, PQ else
    zip: np.ndarray        # float64 [n,6] P_Z, P_I, P_P, Q_Z, Q_I, Q_P (pu at |V|=1)
    p_gen: np.ndarray      # float64 [n] generation (DG); zero without DG
    q_gen: np.ndarray      # float64 [n] (PV nodes: starting value of Q)
    v_mag: np.ndarray      # float64 [n] magnitude set-point of source and PV nodes
    v_ang: np.ndarray      # float64 [n] nominal phase angle of every node
    seed: int = 0
    # delta-connected ZIP loads: node k draws from its phase to node
    # delta_to[k] (another phase of the same bus; -1: none) the load
    # zip_delta[k] (P_Z, P_I, P_P, Q_Z, Q_I, Q_P at the nominal line-to-line
    # voltage sqrt(3) pu)
    delta_to: np.ndarray = None    # int32 [n] or None
    zip_delta: np.ndarray = None   # float64 [n,6] or None

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def with_zip(self, zip_, name=None) -> "CimCase":
        return dataclasses.replace(self, zip=np.ascontiguousarray(zip_, np.float64),
                                   name=name or self.name)


# ----------------------------------------------------------------------------
# helpers


def _stamp_csr(nn, rows, cols, vals):
    """Sum admittance stamps into a sorted CSR with int32 indices."""
    a = sp.coo_matrix((np.asarray(vals, np.complex128),
                       (np.asarray(rows, np.int64), np.asarray(cols, np.int64))),
                      shape=(nn, nn)).tocsr()
    a.sum_duplicates()
    a.sort_indices()
    return (a.indptr.astype(np.int32), a.indices.astype(np.int32),
            a.data.astype(np.complex128))


def _random_recursive_tree(n, rng):
    if n <= 1:
        return np.zeros(0, np.int64)
    u = rng.random(n - 1)
    parents = np.floor(u * np.arange(1, n)).astype(np.int64)
    return parents


def _tree_plus_chords(n, n_extra, rng):
    parents = _random_recursive_tree(n, rng)
    f = list(parents)
    t = list(range(1, n))
    seen = {(min(a, b), max(a, b)) for a, b in zip(f, t)}
    max_pairs = n * (n - 1) // 2
    n_extra = min(n_extra, max_pairs - len(seen))
    added = 0
    while added < n_extra:
        i = int(rng.integers(0, n))
        j = int(rng.integers(0, n))
        if i == j:
            continue
        key = (min(i, j), max(i, j))
        if key in seen:
            continue
        seen.add(key)
        f.append(key[0])
        t.append(key[1])
        added += 1
    return np.asarray(f, np.int32), np.asarray(t, np.int32)


# ----------------------------------------------------------------------------
# single-phase meshed grids


def make_polar_grid(n, n_extra, n_pv, seed, balanced=False, name=None):
    """Seeded single-phase meshed grid (see module docstring)."""
    rng = np.random.default_rng(seed)
    f, t = _tree_plus_chords(n, n_extra, rng)
    m = f.shape[0]
    r = rng.uniform(0.01, 0.05, m)
    x = rng.uniform(0.05, 0.2, m)
    b = rng.uniform(0.0, 0.04, m)

    # nodal admittance stamps (eq. 2-3): series y_ij off the diagonal with a
    # minus sign, y_ij plus the half charging on both diagonals
    ys = 1.0 / (r + 1j * x)
    sh = 0.5j * b
    rows = np.concatenate([f, t, f, t])
    cols = np.concatenate([f, t, t, f])
    vals = np.concatenate([ys + sh, ys + sh, -ys, -ys])
    row_ptr, col, y = _stamp_csr(n, rows, cols, vals)

    bus_type = np.full(n, PQ, np.int8)
    bus_type[0] = SLACK
    n_pv = min(n_pv, n - 1)
    pv = np.sort(rng.choice(np.arange(1, n), size=n_pv, replace=False)) if n_pv else np.zeros(0, int)
    bus_type[pv] = PV
    pq = np.flatnonzero(bus_type == PQ)

    p_gen = np.zeros(n)
    p_gen[pv] = rng.uniform(0.2, 0.8, pv.shape[0])
    p_load = np.zeros(n)
    p_load[pq] = rng.uniform(0.05, 0.3, pq.shape[0])
    if balanced and pv.shape[0] and pq.shape[0]:
        p_gen[pv] *= 0.6
        p_load[pq] *= p_gen.sum() / p_load.sum()
    q_load = p_load * PF_LAG_TAN

    p_sp = p_gen - p_load
    q_sp = -q_load
    v_mag = np.ones(n)
    v_mag[pv] = 1.02
    v_ang = np.zeros(n)
    return PolarCase(name=name or f"grid{n}", n=n, f=f, t=t, r=r, x=x, b=b,
                     row_ptr=row_ptr, col=col, y=y, bus_type=bus_type,
                     p_sp=p_sp, q_sp=q_sp, v_mag=v_mag, v_ang=v_ang, seed=seed)


def perturb_loads(case, seed, lo=0.8, hi=1.2):
    """Scale every load (P and Q together) by a seeded factor U[lo, hi].

    Works on both case kinds: a PolarCase's PQ-bus injections, or the ZIP
    coefficients of a CimCase (one factor per phase-node).
    """
    rng = np.random.default_rng(seed)
    if isinstance(case, PolarCase):
        fac = rng.uniform(lo, hi, case.n)
        load = case.bus_type == PQ
        p = np.where(load, case.p_sp * fac, case.p_sp)
        q = np.where(load, case.q_sp * fac, case.q_sp)
        return case.with_injections(p, q, name=f"{case.name}+p{seed}")
    fac = rng.uniform(lo, hi, case.n)
    return case.with_zip(case.zip * fac[:, None], name=f"{case.name}+p{seed}")


# ----------------------------------------------------------------------------
# three-phase feeders


_SUBSETS_1 = [(0,), (1,), (2,)]
_SUBSETS_2 = [(0, 1), (1, 2), (0, 2)]


def make_feeder(n_bus, seed, laterals=True, lateral_frac=0.20, balanced=False,
                zip_mode="random", load_scale=None, coupling=None, name=None):
    """Seeded three-phase radial feeder (see module docstring).

    ``balanced`` makes every load identical per phase and every branch use the
    same self impedance pattern (used by the balanced-feeder test); ``zip_mode``
    is "random" (Dirichlet fractions), "P", "I" or "Z" (pure load type).
    ``coupling`` fixes k for every branch when given.
    """
    rng = np.random.default_rng(seed)
    if load_scale is None:
        load_scale = FEEDER_LOAD_SCALE
    parents = _random_recursive_tree(n_bus, rng)

    # subtree sizes (children have larger indices than parents)
    size = np.ones(n_bus, np.int64)
    for k in range(n_bus - 1, 0, -1):
        size[parents[k - 1]] += size[k]

    phases = np.ones((n_bus, 3), np.int8)
    if laterals and n_bus > 2:
        children = [[] for _ in range(n_bus)]
        for k in range(1, n_bus):
            children[parents[k - 1]].append(k)

        def subtree(k):
            out, stack = [], [k]
            while stack:
                u = stack.pop()
                out.append(u)
                stack.extend(children[u])
            return out

        cap = max(2, int(0.02 * n_bus))
        order = rng.permutation(np.arange(1, n_bus))
        picks = rng.random(n_bus)
        which = rng.integers(0, 3, n_bus)
        in_lateral = np.zeros(n_bus, bool)
        covered = 0
        target = lateral_frac * n_bus
        for k in order:
            if covered >= target:
                break
            if size[k] > cap or in_lateral[k]:
                continue
            sub = subtree(int(k))
            if in_lateral[sub].any():
                continue  # would swallow an existing lateral
            in_lateral[sub] = True
            covered += len(sub)
            ph = _SUBSETS_1[which[k]] if picks[k] < 0.5 else _SUBSETS_2[which[k]]
            phases[sub] = 0
            phases[np.ix_(sub, list(ph))] = 1

    # branch impedances (per unit)
    m = n_bus - 1
    f = parents.astype(np.int32)
    t = np.arange(1, n_bus, dtype=np.int32)
    zs = rng.uniform(0.3, 0.6, m) + 1j * rng.uniform(0.6, 1.2, m)
    kk = rng.uniform(0.3, 0.5, m) if coupling is None else np.full(m, float(coupling))
    ln = rng.uniform(0.05, 0.5, m)
    if balanced:
        zs[:] = zs[0]
        kk[:] = kk[0]
    eye = np.eye(3)
    ones = np.ones((3, 3))
    zbr = np.empty((m, 3, 3), np.complex128)
    for e in range(m):
        zbr[e] = ln[e] * zs[e] * ((1.0 - kk[e]) * eye + kk[e] * ones) / FEEDER_Z_BASE

    # phase-node numbering: bus-major, phase-minor, present phases only
    node_of = -np.ones((n_bus, 3), np.int64)
    nb, nph = [], []
    for i in range(n_bus):
        for ph in range(3):
            if phases[i, ph]:
                node_of[i, ph] = len(nb)
                nb.append(i)
                nph.append(ph)
    nn = len(nb)
    node_bus = np.asarray(nb, np.int32)
    node_phase = np.asarray(nph, np.int32)

    # admittance stamps (eq. 2-3 with the 3x3 blocks of eq. 11)
    rows, cols, vals = [], [], []
    for e in range(m):
        pa, ch = int(f[e]), int(t[e])
        ph = [q for q in range(3) if phases[ch, q]]
        zsub = zbr[e][np.ix_(ph, ph)]
        ysub = np.linalg.inv(zsub)
        ia = [node_of[pa, q] for q in ph]
        ib = [node_of[ch, q] for q in ph]
        for u in range(len(ph)):
            for v in range(len(ph)):
                yv = ysub[u, v]
                rows += [ia[u], ib[u], ia[u], ib[u]]
                cols += [ia[v], ib[v], ib[v], ia[v]]
                vals += [yv, yv, -yv, -yv]
    row_ptr, col, y = _stamp_csr(nn, rows, cols, vals)

    node_type = np.full(nn, PQ, np.int8)
    node_type[node_bus == 0] = SLACK

    # ZIP loads on every non-source phase-node
    zip_ = np.zeros((nn, 6))
    frac = rng.dirichlet([1.0, 1.0, 1.0], n_bus)  # Z, I, P per bus
    base_kw = rng.uniform(0.5, 1.5, n_bus)
    imb = rng.uniform(0.7, 1.3, nn)
    for k in range(nn):
        i = node_bus[k]
        if i == 0:
            continue
        if balanced:
            p_kw = load_scale * 1.0
        else:
            p_kw = load_scale * base_kw[i] * imb[k]
        p = p_kw / FEEDER_S_PHASE_KVA
        q = p * PF_LAG_TAN
        if zip_mode == "random" and not balanced:
            fz, fi, fp = frac[i]
        else:
            fz, fi, fp = {"Z": (1, 0, 0), "I": (0, 1, 0), "P": (0, 0, 1),
                          "random": (0, 0, 1)}[zip_mode]
        zip_[k] = [fz * p, fi * p, fp * p, fz * q, fi * q, fp * q]

    nominal = np.array([0.0, -2.0 * math.pi / 3.0, 2.0 * math.pi / 3.0])
    v_ang = nominal[node_phase]
    v_mag = np.ones(nn)
    return CimCase(name=name or f"feeder{n_bus}", n_bus=n_bus, n=nn,
                   node_bus=node_bus, node_phase=node_phase, f=f, t=t, zbr=zbr,
                   bus_phases=phases, row_ptr=row_ptr, col=col, y=y,
                   node_type=node_type, zip=zip_, p_gen=np.zeros(nn),
                   q_gen=np.zeros(nn), v_mag=v_mag, v_ang=v_ang, seed=seed)


# ----------------------------------------------------------------------------
# named workloads


def config_case(cfg, seed=None):
    """The three single-instance workloads.

    0: 30-bus meshed grid (41 branches, 5 PV);
    1: 10,000-bus meshed grid (3,000 chords, 1,000 PV, balanced dispatch);
    2: 2,000-bus three-phase radial feeder with ZIP loads.
    """
    s = BASE_SEED + cfg if seed is None else seed
    if cfg == 0:
        return make_polar_grid(30, 12, 5, s, balanced=False, name="grid30")
    if cfg == 1:
        return make_polar_grid(10000, 3000, 1000, s, balanced=True, name="grid10k")
    if cfg == 2:
        return make_feeder(2000, s, name="feeder2k")
    raise ValueError(f"unknown workload {cfg}")


def _loguniform_int(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def c3_scenarios(count=512, seed=None, lo=100, hi=5000):
    """Batched workload: ``count`` scenarios of log-uniform size, each with
    its own topology and a +-20 % per-bus load perturbation."""
    s = BASE_SEED + 3 if seed is None else seed
    rng = np.random.default_rng(s)
    out = []
    for i in range(count):
        n = _loguniform_int(rng, lo, hi)
        base = make_polar_grid(n, int(round(0.3 * n)), max(1, n // 10), s * 1000 + i,
                               balanced=True, name=f"sc{i}_{n}")
        out.append(perturb_loads(base, s * 7919 + i))
    return out


def c4_pool(seed=None, n_polar=32, n_feeder=16):
    """Served workload: a pool of base grids (70 % / 30 % request mix is drawn
    by the load generator); single-phase n ~ log-uniform[1000, 20000], feeders
    of 500-3000 buses."""
    s = BASE_SEED + 4 if seed is None else seed
    rng = np.random.default_rng(s)
    pool = []
    for i in range(n_polar):
        n = _loguniform_int(rng, 1000, 20000)
        pool.append(make_polar_grid(n, int(round(0.3 * n)), max(1, n // 10),
                                    s * 1000 + i, balanced=True, name=f"pool{i}_{n}"))
    for i in range(n_feeder):
        nb = int(rng.integers(500, 3001))
        pool.append(make_feeder(nb, s * 1000 + 100 + i, name=f"poolf{i}_{nb}"))
    return pool


# ----------------------------------------------------------------------------
# replication-scale cases (the construction of Sec. IV)


REPLICA_BLOCK = 30        # buses of the single-phase base block
REPLICA_LINKS = 2         # inter-block links added with every new block
# dispatch of the PV bus that replaces a copy's slack, as a fraction of the
# copy's load: the losses of the balanced base block at its solution (1.21 %
# of its load for the base seed, chosen once), so that the one slack of the
# whole grid does not have to cover every copy's losses through the links
REPLICA_LOSS_FRAC = 0.012
FEEDER_BASE_BUSES = 906   # buses of the three-phase base feeder
# substation branch (source bus to the feeder's first bus) of the one-replica
# feeder, per unit, no coupling; with R replicas it is divided by R so that
# the drop across it stays what it is for one replica
SUBSTATION_Z = 0.0004 + 0.0016j


def replicate_polar(n_blocks, seed, links=REPLICA_LINKS, loss_frac=REPLICA_LOSS_FRAC, base=None,
                    name=None):
    """Single-phase grid of ``n_blocks`` copies of a 30-bus base block.

    Sec. IV builds its large transmission cases by copying a 30-bus case many
    times and joining the copies with random links; each link repeats an
    existing branch of the base block with its ends in two different copies.
    Recipe: the base block is ``make_polar_grid(30, 12, 5, seed,
    balanced=True)`` (41 branches, 5 PV buses: the shape of IEEE-30, whose
    data is not available); copy r numbers its buses 30 r .. 30 r + 29 and
    repeats every base branch and set-point; every copy r >= 1 is joined to
    earlier copies by ``links`` random links: a uniform base branch (i, j)
    with its impedance and charging becomes the branch from bus i of a
    uniform earlier copy q < r to bus j of copy r.  Bus 0 of copy 0 is the
    slack; bus 0 of every other copy (its own slack in the base block) becomes
    one more PV bus at the base slack's |V|, dispatched at ``loss_frac`` of
    the copy's load.  The base block's PV dispatch equals its load (balanced
    block) and that extra dispatch covers about its losses, so the one slack
    and the links carry little net power.
    """
    rng = np.random.default_rng(seed)
    if base is None:
        base = make_polar_grid(REPLICA_BLOCK, 12, 5, seed, balanced=True)
    nb, mb = base.n, base.m
    R = int(n_blocks)
    off = (np.arange(R, dtype=np.int64) * nb)[:, None]
    f = (base.f[None, :] + off).ravel()
    t = (base.t[None, :] + off).ravel()
    r_ = np.tile(base.r, R)
    x_ = np.tile(base.x, R)
    b_ = np.tile(base.b, R)
    if R > 1 and links > 0:
        blk = np.repeat(np.arange(1, R), links)
        q = np.floor(rng.random(blk.shape[0]) * blk).astype(np.int64)
        e = rng.integers(0, mb, blk.shape[0])
        f = np.concatenate([f, base.f[e] + q * nb])
        t = np.concatenate([t, base.t[e] + blk * nb])
        r_ = np.concatenate([r_, base.r[e]])
        x_ = np.concatenate([x_, base.x[e]])
        b_ = np.concatenate([b_, base.b[e]])
    n = R * nb
    f = f.astype(np.int32)
    t = t.astype(np.int32)
    ys = 1.0 / (r_ + 1j * x_)
    sh = 0.5j * b_
    rows = np.concatenate([f, t, f, t])
    cols = np.concatenate([f, t, t, f])
    vals = np.concatenate([ys + sh, ys + sh, -ys, -ys])
    row_ptr, col, y = _stamp_csr(n, rows, cols, vals)

    bus_type = np.tile(base.bus_type, R)
    bus_type[nb::nb] = PV
    p_sp = np.tile(base.p_sp, R)
    q_sp = np.tile(base.q_sp, R)
    block_load = -base.p_sp[base.bus_type == PQ].sum()
    p_sp[nb::nb] = loss_frac * block_load
    q_sp[nb::nb] = 0.0
    v_mag = np.tile(base.v_mag, R)
    v_ang = np.zeros(n)
    return PolarCase(name=name or f"rep{n}", n=n, f=f, t=t, r=r_, x=x_, b=b_,
                     row_ptr=row_ptr, col=col, y=y, bus_type=bus_type,
                     p_sp=p_sp, q_sp=q_sp, v_mag=v_mag, v_ang=v_ang, seed=seed)


def replicate_feeder(n_copies, seed, base=None, z_sub=SUBSTATION_Z, name=None):
    """Three-phase feeder of ``n_copies`` copies of a 906-bus base feeder.

    Sec. IV scales its distribution case by copying every bus below the first
    bus (the one behind the substation transformer) and adjusting the
    transformer so that the voltage drop stays acceptable.  Recipe: the base
    is ``make_feeder(906, seed)`` (the size of the IEEE 906-bus LV feeder,
    whose data is not available); its bus 0 becomes the first bus F (bus 1
    here), fed from a new three-phase source bus (bus 0, the slack) through
    the substation branch Z = ``z_sub`` / R times the 3x3 identity; the base
    buses 1..905 with their branches, phases and ZIP loads are copied R times,
    copy r numbering its buses 2 + 905 r ..; branches of the base leaving its
    bus 0 leave F in every copy.
    """
    if base is None:
        base = make_feeder(FEEDER_BASE_BUSES, seed)
    R = int(n_copies)
    nb0 = base.n_bus
    per = nb0 - 1                       # copied buses per replica
    n_bus = 2 + R * per

    def bus_map(b0, r):
        return np.where(b0 == 0, 1, 2 + r * per + (b0 - 1))

    # branches: substation, then the copies
    fs, ts, zs = [np.zeros(1, np.int64)], [np.ones(1, np.int64)], [np.eye(3)[None] * (z_sub / R)]
    for r in range(R):
        fs.append(bus_map(base.f.astype(np.int64), r))
        ts.append(bus_map(base.t.astype(np.int64), r))
        zs.append(base.zbr)
    f = np.concatenate(fs).astype(np.int32)
    t = np.concatenate(ts).astype(np.int32)
    zbr = np.concatenate(zs).astype(np.complex128)

    phases = np.ones((n_bus, 3), np.int8)
    phases[2:] = np.tile(base.bus_phases[1:], (R, 1))

    # phase-nodes: bus-major, phase-minor; base bus 0 owns base nodes 0..2
    nn0 = base.n
    assert (base.node_bus[:3] == 0).all() and (base.node_bus[3:] > 0).all()
    perm = nn0 - 3
    nn = 6 + R * perm
    node_bus = np.empty(nn, np.int32)
    node_phase = np.empty(nn, np.int32)
    node_bus[:3], node_bus[3:6] = 0, 1
    node_phase[:3] = node_phase[3:6] = np.arange(3)
    rr = np.repeat(np.arange(R, dtype=np.int64), perm)
    node_bus[6:] = 2 + rr * per + (np.tile(base.node_bus[3:], R) - 1)
    node_phase[6:] = np.tile(base.node_phase[3:], R)

    # admittance: every copy's entries of the base Ybus, with base nodes 0..2
    # mapped onto F's nodes 3..5 (its diagonal block sums over the copies),
    # then the substation branch
    rp = base.row_ptr.astype(np.int64)
    brow = np.repeat(np.arange(nn0, dtype=np.int64), np.diff(rp))
    bcol = base.col.astype(np.int64)

    def node_map(k, r):
        return np.where(k < 3, k + 3, 6 + r * perm + (k - 3))

    rows = [node_map(brow, r) for r in range(R)]
    cols = [node_map(bcol, r) for r in range(R)]
    vals = [np.tile(base.y, R)]
    ysub = np.linalg.inv(np.eye(3) * (z_sub / R))
    s_idx = np.repeat(np.arange(3), 3)
    p_idx = np.tile(np.arange(3), 3)
    yv = ysub[s_idx, p_idx]
    rows += [s_idx, s_idx + 3, s_idx, s_idx + 3]
    cols += [p_idx, p_idx + 3, p_idx + 3, p_idx]
    vals += [yv, yv, -yv, -yv]
    row_ptr, col, y = _stamp_csr(nn, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))

    node_type = np.full(nn, PQ, np.int8)
    node_type[:3] = SLACK
    zip_ = np.zeros((nn, 6))
    zip_[6:] = np.tile(base.zip[3:], (R, 1))
    nominal = np.array([0.0, -2.0 * math.pi / 3.0, 2.0 * math.pi / 3.0])
    return CimCase(name=name or f"repfeeder{n_bus}", n_bus=n_bus, n=nn,
                   node_bus=node_bus, node_phase=node_phase, f=f, t=t, zbr=zbr,
                   bus_phases=phases, row_ptr=row_ptr, col=col, y=y,
                   node_type=node_type, zip=zip_, p_gen=np.zeros(nn),
                   q_gen=np.zeros(nn), v_mag=np.ones(nn), v_ang=nominal[node_phase],
                   seed=seed)


REPLICATION_SEED_POLAR = BASE_SEED + 5
REPLICATION_SEED_FEEDER = BASE_SEED + 6
# the feeder sizes of Table 1 are 906 x 1, 2, 4, ..., 256 buses
FEEDER_COPIES = tuple(1 << k for k in range(9))


def replication_feeder_tol(n_copies):
    """Stop tolerance of the replicated feeder with ``n_copies`` copies.

    The first bus joins every copy's top branches (about 7 per copy, ~600 pu
    each) and the substation branch, so its row of Ybus holds terms of ~1e6
    pu that cancel to ~0; the FP64 rounding of that sum at the exact root is
    4.7e-9 at 128 copies and 2.2e-8 at 256.  The 1e-8 pu test holds up to 128
    copies; the 256-copy case stops at 1e-7 pu.
    """
    return 1e-8 if n_copies <= 128 else 1e-7


def replication_polar(n_blocks=1600):
    """The replicated single-phase workload: 1,600 copies of the 30-bus block
    make the 48,000-bus grid of Sec. IV."""
    return replicate_polar(n_blocks, REPLICATION_SEED_POLAR, name=f"rep{REPLICA_BLOCK * n_blocks}")


def replication_feeder(n_copies):
    """The replicated three-phase workload with ``n_copies`` copies of the
    906-bus feeder (Table 1: 1, 2, 4, ..., 256 copies, 0.9K to 230K buses)."""
    return replicate_feeder(n_copies, REPLICATION_SEED_FEEDER,
                            name=f"repfeeder{2 + (FEEDER_BASE_BUSES - 1) * n_copies}")


# ----------------------------------------------------------------------------
# distributed generation and delta-connected loads on a feeder


def add_dg_and_delta(fc, seed, n_dg=3, dg_v=1.0, dg_scale=(1.0, 3.0), delta_frac=0.25,
                     single_phase_dg=True, name=None):
    """A copy of feeder ``fc`` with voltage-controlled generation (PV
    phase-nodes) and delta-connected loads.

    Recipe: ``n_dg`` uniform three-phase buses (not the source) get a
    three-phase generator: every phase-node becomes PV at |V| = ``dg_v`` with
    P_g = U[dg_scale] x the feeder's mean per-phase load P, Q starting at 0;
    with ``single_phase_dg`` one phase-node of a one- or two-phase bus (when
    there is one) gets a single-phase generator the same way.  A fraction
    ``delta_frac`` of the buses with two or more phases (not the source) turn
    their wye loads into delta loads with the same coefficients: phase a
    draws towards b, b towards c, c towards a on a three-phase bus; on a
    two-phase bus the first present phase draws towards the second (the second
    keeps its wye load).
    """
    rng = np.random.default_rng(seed)
    n = fc.n
    node_type = fc.node_type.copy()
    v_mag = fc.v_mag.copy()
    p_gen = fc.p_gen.copy()
    q_gen = np.zeros(n)
    zip_ = fc.zip.copy()
    delta_to = -np.ones(n, np.int32)
    zip_delta = np.zeros((n, 6))
    nodes_of = [np.flatnonzero(fc.node_bus == b) for b in range(fc.n_bus)]
    nph = np.array([len(x) for x in nodes_of])
    mean_p = float(np.mean(fc.zip[fc.node_bus > 0][:, :3].sum(axis=1)))
    three = np.flatnonzero(nph == 3)
    three = three[three > 0]
    dg_buses = rng.choice(three, size=min(n_dg, three.shape[0]), replace=False) if three.size else []
    for b in dg_buses:
        for k in nodes_of[b]:
            node_type[k] = PV
            v_mag[k] = dg_v
            p_gen[k] = rng.uniform(*dg_scale) * mean_p
    if single_phase_dg:
        part = np.flatnonzero((nph == 1) | (nph == 2))
        if part.size:
            k = nodes_of[int(rng.choice(part))][0]
            node_type[k] = PV
            v_mag[k] = dg_v
            p_gen[k] = rng.uniform(*dg_scale) * mean_p
    multi = np.flatnonzero(nph >= 2)
    multi = multi[multi > 0]
    pick = multi[rng.random(multi.shape[0]) < delta_frac]
    for b in pick:
        ks = nodes_of[b]
        pairs = [(ks[0], ks[1]), (ks[1], ks[2]), (ks[2], ks[0])] if len(ks) == 3 else [(ks[0], ks[1])]
        for k, t in pairs:
            delta_to[k] = t
            zip_delta[k] = zip_[k]
            zip_[k] = 0.0
    return dataclasses.replace(fc, name=name or f"{fc.name}+dg", node_type=node_type, v_mag=v_mag,
                               p_gen=p_gen, q_gen=q_gen, zip=zip_, delta_to=delta_to,
                               zip_delta=zip_delta)
