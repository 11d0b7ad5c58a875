"""FP64 reference of the docking scoring function and its ADADELTA local search.

TEST INFRASTRUCTURE ONLY (see the package docstring): only tests, the smoke
check and the benchmark's CPU-baseline leg may use this module.

What the paper fixes and what is read into it
---------------------------------------------
Sec. 2.1 fixes the structure: the receptor is fixed, a ligand pose is the
genotype (position, orientation, one torsion angle per rotatable bond), the
score is a pairwise free-energy force field, the local search is ADADELTA
(a gradient method whose cost is the gradient), and every evaluation needs the
energy, the three Cartesian gradient sums and the torque, the latter feeding
the orientation and torsion gradients. The paper prints no formula for any of
these terms, so the functional forms below are the published ones it cites:
the AutoDock4 free-energy force field (Morris et al. 1998; Huey et al. 2007)
with the Mehler-Solmajer distance-dependent dielectric, and ADADELTA (Zeiler
2012, Algorithm 1). Every reading of a silent or garbled passage is listed in
the design notes; the code states the reading where it is used.

Every floating-point operation here is float64. Arrays are vectorised over
individuals (leading axis n); loops run over torsions or corners only.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass

import numpy as np

# Mehler-Solmajer sigmoidal dielectric eps(r) = A + B / (1 + k exp(-lambda B r)),
# B = eps0 - A (Protein Eng. 4, 1991).
ELEC_SCALE = 332.06363          # kcal A / (mol e^2)
DIEL_A = -8.5525
DIEL_EPS0 = 78.4
DIEL_B = DIEL_EPS0 - DIEL_A
DIEL_K = 7.7839
DIEL_LAMBDA = 0.003627
DESOLV_SIGMA = 3.5               # A, Gaussian width of the desolvation term
QSOLV = 0.01097                  # charge-dependent part of the solvation parameter
R2_MIN = 1.0e-4                  # A^2, lower clamp on squared pair distance
E_CAP = 1.0e5                    # kcal/mol, cap on the 12-6 / 12-10 term
K_OUT = 100.0                    # kcal/mol/A^2, outside-the-box penalty
MIN_GRAPH_DIST = 4               # pairs closer than this in the bond graph are excluded


# ---------------------------------------------------------------------------
# Preparation: moving sets, fragments, pair list (BFS only).
# ---------------------------------------------------------------------------

@dataclass
class Prepared:
    n_atoms: int
    n_torsions: int
    y0: np.ndarray            # [N, 3] reference coords minus centroid
    charge: np.ndarray        # [N]
    cls: np.ndarray           # [N]
    axis: np.ndarray          # [T, 2] (a_k, b_k), a_k on the root side
    moving: np.ndarray        # bool [T, N], moving set M_k
    depth: np.ndarray         # [T], number of other moving sets containing b_k
    frag: np.ndarray          # [N] fragment id (component after cutting rotatable bonds)
    n_frag: int
    pairs: np.ndarray         # [P, 2] (i < j), sorted, original indexing
    pair_hb: np.ndarray       # bool [P], donor-acceptor pair
    # per-pair force-field parameters
    r0: np.ndarray            # [P] A
    eps: np.ndarray           # [P] kcal/mol
    qq: np.ndarray            # [P] ELEC_SCALE * q_i q_j
    dsolv: np.ndarray         # [P] S_i V_j + S_j V_i
    graph_dist: np.ndarray    # [N, N] bond-graph distance


def _norm(v, axis=-1):
    """Euclidean norm along `axis`, kept as a length-1 axis: sqrt(sum v^2).
    (The same reduction np.linalg.norm performs, written with plain ufuncs so
    that the operation tally in oracle.work can run it on counting scalars.)"""
    return np.sqrt(np.sum(v * v, axis=axis, keepdims=True))


def _f64(a):
    """float64 array of `a`; an object array (the counting scalars of the
    operation tally in oracle.work) is passed through unchanged."""
    a = np.asarray(a)
    return a if a.dtype == object else a.astype(np.float64, copy=False)


def _adjacency(n, bonds):
    adj = [[] for _ in range(n)]
    for u, v in bonds:
        adj[int(u)].append(int(v))
        adj[int(v)].append(int(u))
    return adj


def _bfs(adj, start, blocked=None):
    """Distances from `start`; `blocked` is an undirected edge never crossed."""
    n = len(adj)
    dist = np.full(n, -1, dtype=np.int64)
    dist[start] = 0
    dq = deque([start])
    while dq:
        u = dq.popleft()
        for v in adj[u]:
            if blocked is not None and {u, v} == blocked:
                continue
            if dist[v] < 0:
                dist[v] = dist[u] + 1
                dq.append(v)
    return dist


def prepare(lig, ff) -> Prepared:
    """Topology of the ligand from its bond graph (a tree, or a connected
    graph whose rings lie inside rigid fragments).

    Reading (the paper is silent on every item here):
    * torsion k turns the atoms reachable from b_k without crossing the bond,
      where a_k is the end closer to the root atom;
    * fragments are the connected components left after cutting the
      rotatable bonds;
    * intramolecular pairs are (i < j) at bond-graph distance >= 4 that lie in
      different fragments;
    * a pair is a hydrogen-bond pair when one class is a donor and the other an
      acceptor, otherwise a van der Waals pair.
    """
    n = lig.n_atoms
    bonds = np.asarray(lig.bonds, dtype=np.int64).reshape(-1, 2)
    adj = _adjacency(n, bonds)
    root_dist = _bfs(adj, int(lig.root))
    T = int(len(lig.rot_bonds))
    axis = np.zeros((T, 2), dtype=np.int64)
    moving = np.zeros((T, n), dtype=bool)
    for k, bidx in enumerate(lig.rot_bonds):
        u, v = (int(x) for x in bonds[int(bidx)])
        a, b = (u, v) if root_dist[u] < root_dist[v] else (v, u)
        axis[k] = (a, b)
        moving[k] = _bfs(adj, b, blocked={a, b}) >= 0
        if moving[k][a]:
            # a bond in a ring has no side to turn: the torsion is undefined
            raise ValueError(f"rotatable bond {int(bidx)} ({a}-{b}) lies in a ring")
    depth = np.array([sum(moving[j, axis[k, 1]] for j in range(T) if j != k)
                      for k in range(T)], dtype=np.int64)
    # fragments: BFS over non-rotatable bonds
    rot_set = {frozenset((int(bonds[int(b)][0]), int(bonds[int(b)][1]))) for b in lig.rot_bonds}
    frag = np.full(n, -1, dtype=np.int64)
    nf = 0
    for s in range(n):
        if frag[s] >= 0:
            continue
        frag[s] = nf
        dq = deque([s])
        while dq:
            u = dq.popleft()
            for v in adj[u]:
                if frozenset((u, v)) in rot_set or frag[v] >= 0:
                    continue
                frag[v] = nf
                dq.append(v)
        nf += 1
    gdist = np.stack([_bfs(adj, s) for s in range(n)]) if n else np.zeros((0, 0), np.int64)
    ii, jj = np.triu_indices(n, k=1)
    keep = (gdist[ii, jj] >= MIN_GRAPH_DIST) & (frag[ii] != frag[jj])
    pairs = np.stack([ii[keep], jj[keep]], axis=1).astype(np.int64).reshape(-1, 2)
    cls = np.asarray(lig.cls, dtype=np.int64)
    q = np.asarray(lig.charge, dtype=np.float64)
    ci, cj = cls[pairs[:, 0]], cls[pairs[:, 1]]
    don = np.isin(cls, ff.donors)
    acc = np.isin(cls, ff.acceptors)
    hb = (don[pairs[:, 0]] & acc[pairs[:, 1]]) | (acc[pairs[:, 0]] & don[pairs[:, 1]])
    r0 = ff.radius[ci] + ff.radius[cj]
    eps = np.sqrt(ff.eps[ci] * ff.eps[cj])
    # hydrogen-bond parameters by (donor class, acceptor class)
    for p in np.nonzero(hb)[0]:
        a_, b_ = int(ci[p]), int(cj[p])
        d_cls, a_cls = (a_, b_) if a_ in ff.donors else (b_, a_)
        di, ai = ff.donors.index(d_cls), ff.acceptors.index(a_cls)
        r0[p] = ff.hb_r0[di, ai]
        eps[p] = ff.hb_eps[di, ai]
    S = ff.solv[cls] + QSOLV * np.abs(q)
    V = ff.vol[cls]
    i_, j_ = pairs[:, 0], pairs[:, 1]
    dsolv = S[i_] * V[j_] + S[j_] * V[i_]
    qq = ELEC_SCALE * q[i_] * q[j_]
    xyz = np.asarray(lig.xyz, dtype=np.float64)
    y0 = xyz - xyz.mean(axis=0) if n else xyz
    return Prepared(n, T, y0, q, cls, axis, moving, depth, frag, nf, pairs, hb,
                    r0, eps, qq, dsolv, gdist)


# ---------------------------------------------------------------------------
# Genotype -> pose.
# ---------------------------------------------------------------------------

def quat_matrix(q):
    """Active rotation matrix of the unit quaternion (w, x, y, z); q [..., 4]."""
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3), dtype=q.dtype)
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def rodrigues(v, u, ang):
    """Rotate vectors v [..., 3] about unit axes u [..., 3] by ang [...] (right hand)."""
    c = np.cos(ang)[..., None]
    s = np.sin(ang)[..., None]
    return v * c + np.cross(u, v) * s + u * np.sum(u * v, axis=-1, keepdims=True) * (1 - c)


def torsion_order(prep: Prepared):
    """Leaf-first order: decreasing depth (stable in torsion index)."""
    return sorted(range(prep.n_torsions), key=lambda k: (-prep.depth[k], k))


def internal_coords(prep: Prepared, psi):
    """Ligand-frame coordinates after the torsions; psi [n, T] -> [n, N, 3].

    Reading: each torsion turns its moving set by +psi_k (right-hand rule
    about the direction a_k -> b_k) relative to the reference conformation.
    Torsions are applied deepest first, so no axis has moved before it is
    used; this is the same conformation as root-first with current axes.
    """
    n = psi.shape[0]
    y = np.broadcast_to(prep.y0, (n, prep.n_atoms, 3)).astype(np.result_type(prep.y0, psi))
    for k in torsion_order(prep):
        a, b = prep.axis[k]
        p = y[:, a, :]
        u = y[:, b, :] - p
        u = u / _norm(u)
        M = prep.moving[k]
        rel = y[:, M, :] - p[:, None, :]
        y[:, M, :] = rodrigues(rel, u[:, None, :], np.repeat(psi[:, k:k + 1], M.sum(), axis=1)) \
            + p[:, None, :]
    return y


def pose(prep: Prepared, genotypes):
    """World coordinates x_i = R(q/|q|) y_i + t; genotypes [n, 7+T] -> [n, N, 3]."""
    g = _f64(genotypes)
    t = g[:, 0:3]
    q = g[:, 3:7]
    qh = q / _norm(q, axis=1)
    y = internal_coords(prep, g[:, 7:])
    R = quat_matrix(qh)
    return np.einsum('nab,nib->nia', R, y) + t[:, None, :]


# ---------------------------------------------------------------------------
# Intermolecular term: trilinear interpolation of the grid maps.
# ---------------------------------------------------------------------------

def box_bounds(dims, origin, spacing):
    lo = np.asarray(origin, dtype=np.float64)
    hi = lo + (np.asarray(dims, dtype=np.float64) - 1) * spacing
    return lo, hi


def trilinear(mp, origin, spacing, x):
    """Value and gradient of the trilinear interpolant of one map.

    mp [nz, ny, nx] (x fastest), x [..., 3] in A. Reading for points outside
    the box: the interpolant is evaluated at the point clamped into the box
    and its gradient is zero along clamped axes. Cells: c = clamp(floor(u), 0,
    n-2), f = u - c, with u = (x - origin)/h. The gradient is the exact
    derivative of the interpolant (per-axis derivative of the weights) / h.
    """
    nz, ny, nx = mp.shape
    dims = np.array([nx, ny, nz])
    lo, hi = box_bounds(dims, origin, spacing)
    xc = np.clip(x, lo, hi)
    inside_axis = (x == xc)
    u = (xc - lo) / spacing
    c = np.clip(np.floor(u), 0, dims - 2).astype(np.int64)
    f = u - c
    val = np.zeros(x.shape[:-1], dtype=x.dtype)
    dval = np.zeros(x.shape, dtype=x.dtype)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                v = mp[c[..., 2] + dz, c[..., 1] + dy, c[..., 0] + dx].astype(np.float64)
                wx = f[..., 0] if dx else 1 - f[..., 0]
                wy = f[..., 1] if dy else 1 - f[..., 1]
                wz = f[..., 2] if dz else 1 - f[..., 2]
                sx = 1.0 if dx else -1.0
                sy = 1.0 if dy else -1.0
                sz = 1.0 if dz else -1.0
                val += wx * wy * wz * v
                dval[..., 0] += sx * wy * wz * v
                dval[..., 1] += wx * sy * wz * v
                dval[..., 2] += wx * wy * sz * v
    grad = dval / spacing * inside_axis
    return val, grad


def outside_penalty(x, dims, origin, spacing):
    """K_out * |x - clamp(x)|^2 and its gradient (reading: C^1 at the box face)."""
    lo, hi = box_bounds(dims, origin, spacing)
    d = x - np.clip(x, lo, hi)
    return K_OUT * np.sum(d * d, axis=-1), 2.0 * K_OUT * d


def inter_terms(prep: Prepared, grd, x):
    """Per-atom intermolecular energy e_i [n, N] and gradient [n, N, 3].

    e_i = I(map[cls_i]) + q_i I(map_e) + |q_i| I(map_d) + penalty, where the
    electrostatic and desolvation maps are the last two maps of the set and
    the type maps come first (reading: extra type maps are resident, unused).
    """
    maps = grd.maps
    M = maps.shape[0]
    e_map, d_map = M - 2, M - 1
    n, N, _ = x.shape
    e = np.zeros((n, N), dtype=x.dtype)
    g = np.zeros((n, N, 3), dtype=x.dtype)
    for i in range(N):
        xi = x[:, i, :]
        v, gv = trilinear(maps[int(prep.cls[i])], grd.origin, grd.spacing, xi)
        ve, ge = trilinear(maps[e_map], grd.origin, grd.spacing, xi)
        vd, gd = trilinear(maps[d_map], grd.origin, grd.spacing, xi)
        qi = prep.charge[i]
        e[:, i] = v + qi * ve + abs(qi) * vd
        g[:, i, :] = gv + qi * ge + abs(qi) * gd
    pen, gpen = outside_penalty(x, grd.dims, grd.origin, grd.spacing)
    return e + pen, g + gpen


# ---------------------------------------------------------------------------
# Intramolecular pair terms.
# ---------------------------------------------------------------------------

def dielectric(r):
    """Mehler-Solmajer eps(r) and d eps / dr."""
    ex = np.exp(-DIEL_LAMBDA * DIEL_B * r)
    den = 1.0 + DIEL_K * ex
    eps = DIEL_A + DIEL_B / den
    deps = DIEL_B * DIEL_K * DIEL_LAMBDA * DIEL_B * ex / den ** 2
    return eps, deps


def pair_energy(r2_raw, r0, eps, hb, qq, dsolv):
    """Energy of each listed pair and w = (dE/dr)/r, from the squared distance.

    * r^2 is clamped below at 1e-4 A^2 (w = 0 where clamped);
    * van der Waals 12-6: eps (s^12 - 2 s^6), s = r0/r;
      hydrogen bond 12-10: eps (5 s^12 - 6 s^10); either capped at +1e5
      (no gradient where capped);
    * electrostatics: qq / (r eps(r));
    * desolvation: dsolv exp(-r^2 / (2 sigma^2)).
    Returns (E_total, w, E_lj, E_elec, E_desolv).
    """
    clamped = r2_raw < R2_MIN
    r2 = np.maximum(r2_raw, R2_MIN)
    r = np.sqrt(r2)
    s = r0 / r
    # 12-6 on the van der Waals pairs, 12-10 on the hydrogen-bond pairs (each
    # form evaluated on its own pairs only)
    hbm = np.broadcast_to(hb, r.shape)
    vdw = ~hbm
    epsb = np.broadcast_to(eps, r.shape)
    e_lj = np.zeros_like(r)
    de_lj = np.zeros_like(r)
    sv, ev, rv = s[vdw], epsb[vdw], r[vdw]
    s2 = sv * sv
    s6 = s2 * s2 * s2
    s12 = s6 * s6
    e_lj[vdw] = ev * (s12 - 2.0 * s6)
    de_lj[vdw] = ev * (-12.0 * s12 + 12.0 * s6) / rv
    sh, eh, rh = s[hbm], epsb[hbm], r[hbm]
    s2 = sh * sh
    s6 = s2 * s2 * s2
    s10 = s6 * s2 * s2
    s12 = s6 * s6
    e_lj[hbm] = eh * (5.0 * s12 - 6.0 * s10)
    de_lj[hbm] = eh * (-60.0 * s12 + 60.0 * s10) / rh
    capped = e_lj > E_CAP
    e_lj = np.where(capped, E_CAP, e_lj)
    de_lj = np.where(capped, 0.0, de_lj)
    de, dde = dielectric(r)
    e_el = qq / (r * de)
    de_el = -qq * (de + r * dde) / (r * de) ** 2
    gs = np.exp(-r2 / (2.0 * DESOLV_SIGMA ** 2))
    e_ds = dsolv * gs
    de_ds = e_ds * (-r / DESOLV_SIGMA ** 2)
    w = (de_lj + de_el + de_ds) / r
    w = np.where(clamped, 0.0, w)
    return e_lj + e_el + e_ds, w, e_lj, e_el, e_ds


def intra_terms(prep: Prepared, x, with_abs: bool = False):
    """Sum of pair energies [n] and per-atom intramolecular gradient [n, N, 3].

    With `with_abs`, also returns the sum of the magnitudes of the pair
    energies [n] (the scale against which rounding of the sum is judged).
    """
    n, N, _ = x.shape
    i, j = prep.pairs[:, 0], prep.pairs[:, 1]
    d = x[:, j, :] - x[:, i, :]
    r2 = np.sum(d * d, axis=-1)
    e, w, *_ = pair_energy(r2, prep.r0, prep.eps, prep.pair_hb, prep.qq, prep.dsolv)
    f = w[..., None] * d                        # dE/dx_j for each pair
    g = np.zeros((n, N, 3), dtype=x.dtype)
    np.add.at(g, (slice(None), j), f)
    np.add.at(g, (slice(None), i), -f)
    if with_abs:
        return e.sum(axis=1), g, np.abs(e).sum(axis=1)
    return e.sum(axis=1), g


def intra_terms_bruteforce(prep: Prepared, x):
    """O(N^2) double loop over atom pairs; used as a pin for intra_terms."""
    n, N, _ = x.shape
    listed = {(int(a), int(b)): p for p, (a, b) in enumerate(prep.pairs)}
    E = np.zeros(n)
    g = np.zeros((n, N, 3))
    for a in range(N):
        for b in range(a + 1, N):
            if (a, b) not in listed:
                continue
            p = listed[(a, b)]
            d = x[:, b, :] - x[:, a, :]
            r2 = np.sum(d * d, axis=-1)
            e, w, *_ = pair_energy(r2, prep.r0[p], prep.eps[p], prep.pair_hb[p],
                                   prep.qq[p], prep.dsolv[p])
            E += e
            g[:, b, :] += w[:, None] * d
            g[:, a, :] -= w[:, None] * d
    return E, g


# ---------------------------------------------------------------------------
# Gradient -> genotype.
# ---------------------------------------------------------------------------

def quat_mul(a, b):
    """Hamilton product of quaternions (w, x, y, z), broadcasting over [..., 4]."""
    aw, av = a[..., :1], a[..., 1:]
    bw, bv = b[..., :1], b[..., 1:]
    w = aw * bw - np.sum(av * bv, axis=-1, keepdims=True)
    v = aw * bv + bw * av + np.cross(av, bv)
    return np.concatenate([w, v], axis=-1)


def genotype_gradient(prep: Prepared, genotypes, x, g):
    """dE/d(genotype) from world coordinates x and per-atom gradients g.

    * translation: sum_i g_i;
    * orientation: torque tau = sum_i (x_i - t) x g_i is the gradient with
      respect to a world-frame rotation vector; for q = |q| q_hat the gradient
      is (2/|q|) ((0, tau) (x) q_hat), orthogonal to q;
    * torsion k: u_k . sum_{i in M_k} (x_i - x_{a_k}) x g_i, with u_k the unit
      world-frame bond direction a_k -> b_k (the torque about the bond).
    """
    gen = _f64(genotypes)
    n = gen.shape[0]
    t = gen[:, 0:3]
    q = gen[:, 3:7]
    qn = _norm(q, axis=1)
    qh = q / qn
    out = np.zeros((n, 7 + prep.n_torsions), dtype=g.dtype)
    out[:, 0:3] = g.sum(axis=1)
    tau = np.cross(x - t[:, None, :], g).sum(axis=1)
    tq = np.concatenate([np.zeros((n, 1), dtype=tau.dtype), tau], axis=1)
    out[:, 3:7] = 2.0 / qn * quat_mul(tq, qh)
    for k in range(prep.n_torsions):
        a, b = prep.axis[k]
        u = x[:, b, :] - x[:, a, :]
        u = u / _norm(u)
        M = prep.moving[k]
        tk = np.cross(x[:, M, :] - x[:, a, None, :], g[:, M, :]).sum(axis=1)
        out[:, 7 + k] = np.sum(u * tk, axis=-1)
    return out


@dataclass
class ScoreResult:
    energy: np.ndarray        # [n]
    grad: np.ndarray          # [n, G]
    x: np.ndarray             # [n, N, 3]
    atom_grad: np.ndarray     # [n, N, 3]
    e_inter: np.ndarray       # [n, N] per-atom intermolecular energy
    e_intra: np.ndarray       # [n]
    torque: np.ndarray        # [n, 3]
    e_abs: np.ndarray         # [n] sum of |per-atom| and |per-pair| energy terms


def score(prep: Prepared, grd, genotypes) -> ScoreResult:
    """Energy and analytic gradient of each genotype (one scoring evaluation)."""
    gen = _f64(genotypes)
    x = pose(prep, gen)
    e_in, g_in = inter_terms(prep, grd, x)
    e_ia, g_ia, a_ia = intra_terms(prep, x, with_abs=True)
    gat = g_in + g_ia
    E = e_in.sum(axis=1) + e_ia
    grad = genotype_gradient(prep, gen, x, gat)
    tau = np.cross(x - gen[:, None, 0:3], gat).sum(axis=1)
    return ScoreResult(E, grad, x, gat, e_in, e_ia, tau, np.abs(e_in).sum(axis=1) + a_ia)


# ---------------------------------------------------------------------------
# ADADELTA local search.
# ---------------------------------------------------------------------------

@dataclass
class LSState:
    genotype: np.ndarray      # [n, G] current point x_t
    acc_g2: np.ndarray        # [n, G] running E[g^2]
    acc_dx2: np.ndarray       # [n, G] running E[dx^2]
    best_genotype: np.ndarray  # [n, G]
    best_energy: np.ndarray   # [n]
    energy: np.ndarray        # [n] energy at the last evaluated point
    iters_done: np.ndarray    # [n] int


def ls_init(genotypes) -> LSState:
    g = np.asarray(genotypes, dtype=np.float64).copy()
    n = g.shape[0]
    return LSState(g, np.zeros_like(g), np.zeros_like(g), g.copy(),
                   np.full(n, np.inf), np.full(n, np.nan), np.zeros(n, dtype=np.int64))


def adadelta_step(x, grad, acc_g2, acc_dx2, rho, eps):
    """One ADADELTA update (Zeiler 2012, Alg. 1), elementwise over all genes.

    Reading of the paper's update (Sec. 2.1, printed with a + sign): the step
    descends, dx = -RMS[dx]_{t-1} / RMS[g]_t * g with eps inside both roots.
    The quaternion is renormalised afterwards (kept if its norm collapses
    below 1e-6); its accumulators are left as updated.
    Returns (x_new, acc_g2, acc_dx2).
    """
    acc_g2 = rho * acc_g2 + (1.0 - rho) * grad * grad
    dx = -np.sqrt(acc_dx2 + eps) / np.sqrt(acc_g2 + eps) * grad
    acc_dx2 = rho * acc_dx2 + (1.0 - rho) * dx * dx
    xn = x + dx
    q = xn[:, 3:7]
    nq = _norm(q, axis=1)
    ok = nq[:, 0] >= 1e-6
    xn[ok, 3:7] = q[ok] / nq[ok]
    xn[~ok, 3:7] = x[~ok, 3:7]
    return xn, acc_g2, acc_dx2


def _track_best(st: LSState, E, x):
    better = E < st.best_energy          # strict: the first minimum wins ties
    st.best_energy = np.where(better, E, st.best_energy)
    st.best_genotype = np.where(better[:, None], x, st.best_genotype)


def local_search(prep: Prepared, grd, state: LSState, iterations: int,
                 rho: float = 0.8, eps: float = 1e-2, final_eval: bool = True,
                 trace=None) -> LSState:
    """ADADELTA local search over every individual, in place on `state`.

    Each iteration evaluates E and its gradient at the current point, records
    the point if it is the best seen, and takes one ADADELTA step. With
    `final_eval` the point reached after the last step is evaluated too, so
    300 iterations cost 301 evaluations. `trace`, if a list, receives
    (x_t, E_t, grad_t) for every evaluation.
    """
    st = state
    for _ in range(iterations):
        r = score(prep, grd, st.genotype)
        if trace is not None:
            trace.append((st.genotype.copy(), r.energy.copy(), r.grad.copy()))
        st.energy = r.energy
        _track_best(st, r.energy, st.genotype)
        st.genotype, st.acc_g2, st.acc_dx2 = adadelta_step(
            st.genotype, r.grad, st.acc_g2, st.acc_dx2, rho, eps)
        st.iters_done = st.iters_done + 1
    if final_eval:
        r = score(prep, grd, st.genotype)
        if trace is not None:
            trace.append((st.genotype.copy(), r.energy.copy(), r.grad.copy()))
        st.energy = r.energy
        _track_best(st, r.energy, st.genotype)
    return st


def count_work(prep: Prepared):
    """Sizes that fix the algorithmic work of one evaluation."""
    return {"atoms": prep.n_atoms, "torsions": prep.n_torsions,
            "pairs": int(prep.pairs.shape[0]), "genes": 7 + prep.n_torsions,
            "hb_pairs": int(prep.pair_hb.sum())}
