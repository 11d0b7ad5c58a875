"""Shared pieces of the GPU parity tests: tolerances and oracle comparisons.

How a GPU result is compared with the FP64 oracle
-------------------------------------------------
* Pose: the kernel's atom positions come back through the per-atom debug
  output (each atom's position relative to the translation genes, in the
  FP32 the kernel holds); t + that position, summed in FP64, is the world
  position the kernel's grid and pair terms use. It is checked against the
  oracle's pose of the same genotype (POSE_TOL).
* Energy and gradient: the oracle is evaluated at exactly those positions,
  so the comparison measures the kernel's arithmetic from a given pose,
  without the FP32 rounding of the pose itself (which alone moves E by about
  u * sum_i |g_i| |x_i|, more than 1e-5 of |E| at clashes). The bounds are
  the FP32 path's: |dE| <= 1e-5 max(|E|, 1), ||dg|| <= 1e-4 max(||g||, 1).
* Conditioning: when E is a small difference of large terms, the rounding of
  the terms themselves (~2^-24 of each) exceeds 1e-5 of |E|; and a steep term
  amplifies the rounding of its own argument in FP32: a pair energy moves by
  |r dE/dr| times the relative rounding of its separation (the difference of
  two FP32 positions, squared and summed, then rsq: about 2u), a grid energy
  by h |grad e| times the rounding of its cell fraction (about 1.5u per
  axis). An individual may then pass by |dE| <= COND_TOL * (sum of the terms'
  magnitudes) + SENS_TOL * (sum over pairs of |r dE/dr| + h * sum over atoms
  of the 1-norm of the grid gradient); at most COND_CAP of the individuals of
  a check may, and the count is printed.
* Kinks: the score is only piecewise smooth (trilinear cells change at grid
  faces, the box clamp at the box faces, the 12-6/12-10 term at its cap, the
  r^2 clamp). An atom within rounding reach of a kink may take the other
  side in FP32; its energy is continuous there (checked strictly), its
  gradient is not. Such individuals (at most KINK_CAP of a check) are
  exempt from the gradient bound only, and counted.
"""
from dataclasses import dataclass

import numpy as np

E_TOL = 1e-5
G_TOL = 1e-4
POSE_TOL = 1e-4            # A, world coordinates
COND_TOL = 2.0 ** -20      # |dE| bound relative to the sum of the terms' magnitudes
SENS_TOL = 2.0 ** -22      # |dE| bound relative to the terms' sensitivity to their arguments' rounding
COND_CAP = 0.01            # share of a check's individuals that may pass only by COND_TOL / SENS_TOL
KINK_CAP = 0.03            # share of a check's individuals that may sit at a kink
FACE_TOL_U = 2e-5          # cell units: rounding reach of a cell face (|x| <= 20 A, u <= 95)
BOX_TOL = 1e-5             # A: rounding reach of a box face
CAP_TOL = 1e-5             # relative distance of a 12-6/12-10 energy to its cap
# error of the half-width split reductions per element (2-term BF16 keeps 16
# significant bits; the others reach FP32 level)
SPLIT_U = {0: 0.0, 1: 0.0, 2: 2.0 ** -16, 3: 2.0 ** -22, 4: 2.0 ** -24}


def e_relerr(e_gpu, e_ref):
    e_gpu = np.asarray(e_gpu, np.float64)
    e_ref = np.asarray(e_ref, np.float64)
    return np.abs(e_gpu - e_ref) / np.maximum(np.abs(e_ref), 1.0)


def g_relerr(g_gpu, g_ref):
    g_gpu = np.asarray(g_gpu, np.float64)
    g_ref = np.asarray(g_ref, np.float64)
    return np.linalg.norm(g_gpu - g_ref, axis=-1) / np.maximum(np.linalg.norm(g_ref, axis=-1), 1.0)


def world_positions(genotypes, atom_out):
    """World positions the kernel used: t + (x - t), summed in FP64."""
    gen = np.asarray(genotypes, np.float32).astype(np.float64)
    rel = np.asarray(atom_out, np.float32)[:, :, 0:3].astype(np.float64)
    return gen[:, None, 0:3] + rel


def oracle_at(prep, grd, genotypes, x):
    """The oracle's score of each genotype with its atoms at x [n, N, 3]."""
    from oracle import dock_ref as R
    gen = np.asarray(genotypes, np.float64)
    e_in, g_in = R.inter_terms(prep, grd, x)
    e_ia, g_ia, a_ia = R.intra_terms(prep, x, with_abs=True)
    gat = g_in + g_ia
    grad = R.genotype_gradient(prep, gen, x, gat)
    tau = np.cross(x - gen[:, None, 0:3], gat).sum(axis=1)
    return R.ScoreResult(e_in.sum(axis=1) + e_ia, grad, x, gat, e_in, e_ia, tau,
                         np.abs(e_in).sum(axis=1) + a_ia)


def interp_magnitude(prep, grd, x):
    """Per individual, the sum over atoms of the magnitudes of the terms the
    grid interpolation adds: sum_c w_c (|v_type,c| + |q| |v_elec,c| +
    |q| |v_desolv,c|) over the eight corners c (the interpolant of |map|)."""
    from oracle import dock_ref as R
    maps = np.abs(np.asarray(grd.maps, np.float64))
    M = maps.shape[0]
    out = np.zeros(x.shape[0])
    for i in range(x.shape[1]):
        xi = x[:, i, :]
        aq = abs(float(prep.charge[i]))
        out += R.trilinear(maps[int(prep.cls[i])], grd.origin, grd.spacing, xi)[0]
        out += aq * R.trilinear(maps[M - 2], grd.origin, grd.spacing, xi)[0]
        out += aq * R.trilinear(maps[M - 1], grd.origin, grd.spacing, xi)[0]
    return out


def argument_sensitivity(prep, grd, x):
    """Per individual: sum over pairs of |r dE/dr| plus h times the sum over
    atoms of the 1-norm of the grid term's gradient, at positions x."""
    from oracle import dock_ref as R
    _, g_in = R.inter_terms(prep, grd, x)
    out = grd.spacing * np.abs(g_in).sum(axis=(1, 2))
    if prep.pairs.shape[0]:
        d = x[:, prep.pairs[:, 1]] - x[:, prep.pairs[:, 0]]
        r2 = np.sum(d * d, axis=-1)
        _, w, *_ = R.pair_energy(r2, prep.r0, prep.eps, prep.pair_hb, prep.qq, prep.dsolv)
        out = out + np.abs(w * r2).sum(axis=1)
    return out


def kink_mask(prep, grd, x):
    """Individuals with an atom within rounding reach of a kink of the score.

    Cell faces count only for atoms inside the box (outside, the clamped
    axis has no cell choice to make); box faces only within BOX_TOL of the
    face; the 12-6/12-10 cap within CAP_TOL; the r^2 clamp within 1e-3 of it.
    Returns a boolean mask [n].
    """
    from oracle import dock_ref as R
    dims = np.array(grd.dims, dtype=np.float64)
    lo = np.asarray(grd.origin, np.float64)
    hi = lo + (dims - 1) * grd.spacing
    inside = (x >= lo) & (x <= hi)
    u = (x - lo) / grd.spacing
    frac = np.abs(u - np.round(u))
    face = np.any(inside & (frac < FACE_TOL_U), axis=(1, 2))
    boxf = np.any((np.abs(x - lo) < BOX_TOL) | (np.abs(x - hi) < BOX_TOL), axis=(1, 2))
    if prep.pairs.shape[0] == 0:
        return face | boxf
    i, j = prep.pairs[:, 0], prep.pairs[:, 1]
    d = x[:, j] - x[:, i]
    r2 = np.sum(d * d, axis=-1)
    s = prep.r0 / np.sqrt(np.maximum(r2, R.R2_MIN))
    s6 = s ** 6
    raw = np.where(prep.pair_hb, prep.eps * (5 * s6 * s6 - 6 * s6 * s ** 4), prep.eps * (s6 * s6 - 2 * s6))
    cap = np.any(np.abs(raw - R.E_CAP) < CAP_TOL * R.E_CAP, axis=1)
    clamp = np.any(np.abs(r2 - R.R2_MIN) < 1e-3 * R.R2_MIN, axis=1)
    return face | boxf | cap | clamp


@dataclass
class Report:
    n: int
    pose_err: float           # A, max over atoms
    e_err: np.ndarray         # per individual |dE| / max(|E|, 1)
    g_err: np.ndarray         # per individual ||dg|| / max(||g||, 1) (zeros if no gradient)
    cond: np.ndarray          # E passed only by the conditioning bound
    split: np.ndarray         # E or g passed only by the split reduction's bound
    kink: np.ndarray          # at a kink: gradient exempt
    g_ok: np.ndarray          # gradient within its bound (FP32, or the split's)
    ref: object


def check(tag, prep, grd, genotypes, energy, grad, atom_out, variant=0, cond_cap=COND_CAP,
          kink_cap=KINK_CAP, assert_ok=True):
    """Compare kernel energies (and gradients, if given) with the oracle at
    the kernel's own positions; print the counts; assert the bounds above.

    `variant` selects the reduction's error model. The 2-term BF16 split
    keeps 16 significant bits of each lane's partial sums, so besides the
    FP32 bounds an individual may pass with |dE| <= 2^-16 * (sum of the
    terms' magnitudes) + 1e-5 max(|E|, 1), and with each translation
    gradient component (the only part of g that goes through the split)
    within 2^-16 * sum_i |g_i,c| + 1e-4 max(||g||, 1); such individuals are
    counted, not capped (the bound is the split's own).
    """
    from oracle import dock_ref as R
    gen = np.asarray(genotypes, np.float32)
    n = gen.shape[0]
    E = np.asarray(energy, np.float64)
    x = world_positions(gen, atom_out)
    pose_ref = R.pose(prep, gen.astype(np.float64))
    pose_err = float(np.abs(x - pose_ref).max()) if n else 0.0
    ref = oracle_at(prep, grd, gen, x)
    dE = np.abs(E - ref.energy)
    escale = np.maximum(np.abs(ref.energy), 1.0)
    ee = dE / escale
    strict = ee <= E_TOL
    sens = argument_sensitivity(prep, grd, x) if (~strict).any() else np.zeros(n)
    cond = (~strict) & (dE <= COND_TOL * ref.e_abs + SENS_TOL * sens)
    su = SPLIT_U.get(variant, 0.0)
    coarse = su > COND_TOL
    split = (~strict) & (~cond) & (dE <= su * ref.e_abs + E_TOL * escale) if coarse else np.zeros(n, bool)
    kink = kink_mask(prep, grd, x)
    g_ok = np.ones(n, bool)
    if grad is not None:
        g = np.asarray(grad, np.float64)
        ge = g_relerr(g, ref.grad)
        g_ok = ge <= G_TOL
        if coarse:
            gscale = np.maximum(np.linalg.norm(ref.grad, axis=-1), 1.0)
            gsum = np.abs(ref.atom_grad).sum(axis=1)                    # [n, 3]
            t_ok = np.all(np.abs(g[:, 0:3] - ref.grad[:, 0:3]) <= su * gsum + G_TOL * gscale[:, None], axis=1)
            r_ok = np.linalg.norm(g[:, 3:] - ref.grad[:, 3:], axis=-1) <= G_TOL * gscale
            by_split = (~g_ok) & t_ok & r_ok
            split |= by_split
            g_ok |= by_split
    else:
        ge = np.zeros(n)
    rep = Report(n, pose_err, ee, ge, cond, split, kink, g_ok, ref)
    if n:
        kappa = ref.e_abs / escale
        print(f"\n[{tag}] n={n} pose err {pose_err:.2e} A; E err p50 {np.median(ee):.2e} max {ee.max():.2e}; "
              f"over 1e-5 {int((~strict).sum())} (held to the conditioning bound {int(cond.sum())}"
              + (f", to the split bound {int(split.sum())}" if coarse else "")
              + f"; kappa max {kappa.max():.1f}); g err p50 {np.median(ge):.2e} max {ge.max():.2e} "
              f"(at a kink {int(kink.sum())}, their g err max {ge[kink].max() if kink.any() else 0.0:.2e})",
              flush=True)
    bad = ~(strict | cond | split)
    if bad.any():
        ia = interp_magnitude(prep, grd, x[bad])
        for k, b in enumerate(np.nonzero(bad)[0][:8]):
            print(f"[{tag}] E outside the bounds: individual {b}: E {E[b]:.9g} oracle {ref.energy[b]:.9g} "
                  f"|dE| {dE[b]:.3e}; term magnitudes {ref.e_abs[b]:.6g}; grid interpolation magnitudes "
                  f"{ia[k]:.6g}; argument sensitivity {sens[b]:.6g}", flush=True)
    if assert_ok and n:
        assert pose_err <= POSE_TOL, (tag, pose_err)
        assert not bad.any(), (tag, "E", np.nonzero(bad)[0][:8], ee[bad][:8])
        assert cond.mean() <= cond_cap, (tag, "conditioning share", cond.mean())
        assert kink.mean() <= kink_cap, (tag, "kink share", kink.mean())
        gbad = ~g_ok & ~kink
        assert not gbad.any(), (tag, "g", np.nonzero(gbad)[0][:8], ge[gbad][:8])
    return rep


def gpu_points(dk, grids, ligand, genotypes, variant=0):
    """The kernel's energy, gradient and per-atom output at given genotypes
    (one scoring evaluation each, the given reduction variant)."""
    import torch
    gt = torch.from_numpy(np.ascontiguousarray(genotypes, np.float32)).cuda()
    E, g, ao = dk.score_batch(grids, ligand, gt, variant=variant, atom_out=True)
    torch.cuda.synchronize()
    return E.cpu().numpy(), g.cpu().numpy(), ao.cpu().numpy()


def check_reported(tag, dk, grids, ligand, prep, grd, genotypes, energy, variant=0, exact_rescore=True,
                   **kw):
    """Energies reported by a search kernel (best or last points) against the
    oracle at the kernel's own positions, taken from one scoring evaluation
    of the same genotypes. With `exact_rescore` the scoring kernel must give
    the same FP32 energy, bit for bit (same evaluation code); the reported
    energies themselves are then checked."""
    E_s, g_s, ao = gpu_points(dk, grids, ligand, genotypes, variant)
    rep_e = np.asarray(energy, np.float32)
    same = rep_e.view(np.uint32) == E_s.astype(np.float32).view(np.uint32)
    print(f"\n[{tag}] reported energies equal to a rescoring, bit for bit: {int(same.sum())} of {len(same)}",
          flush=True)
    if exact_rescore:
        assert same.all(), (tag, np.nonzero(~same)[0][:8])
    return check(tag, prep, grd, genotypes, rep_e, None, ao, variant=variant, **kw)


def assert_reports(tag, reports, cond_cap=COND_CAP, kink_cap=KINK_CAP):
    """The bounds of `check` over several checks taken with assert_ok=False
    (for example one per ligand of a batch): caps apply to the total."""
    _E, _G = E_TOL, G_TOL
    n = sum(r.n for r in reports)
    if n == 0:
        return
    pose = max(r.pose_err for r in reports)
    ee = np.concatenate([r.e_err for r in reports])
    ge = np.concatenate([r.g_err for r in reports])
    cond = np.concatenate([r.cond for r in reports])
    split = np.concatenate([r.split for r in reports])
    kink = np.concatenate([r.kink for r in reports])
    print(f"\n[{tag}] total n={n}: pose err {pose:.2e} A; E err max {ee.max():.2e}, over 1e-5 "
          f"{int((ee > _E).sum())} (conditioning bound {int(cond.sum())}, split bound {int(split.sum())}); "
          f"g err max {ge.max():.2e}; at a kink {int(kink.sum())}", flush=True)
    assert pose <= POSE_TOL, (tag, pose)
    assert np.all((ee <= _E) | cond | split), (tag, "E", ee.max())
    assert cond.mean() <= cond_cap, (tag, "conditioning share", cond.mean())
    assert kink.mean() <= kink_cap, (tag, "kink share", kink.mean())
    g_ok = np.concatenate([r.g_ok for r in reports])
    assert np.all(g_ok | kink), (tag, "g", ge[~g_ok & ~kink].max())
