"""Shared pieces of the GPU parity tests: tolerances and oracle comparisons."""
import numpy as np

# FP32 path tolerances (per individual): |dE| / max(|E|, 1) and
# ||dg||_2 / max(||g||_2, 1), against the FP64 oracle at the same genotype.
E_TOL = 1e-5
G_TOL = 1e-4


# Two ill-conditioned cases in which no FP32 evaluation can hold 1e-5
# relative to |E|, each held to the error FP32 itself implies, and counted:
# * E a small difference of large terms (kappa = sum|e_i| / |E| large): the
#   terms' own rounding is ~1e-7 of their magnitude -> E_ABS_TOL * sum|e_i|;
# * E dominated by steep terms (clashes: a 12-6 term moves by 12 dr / r), where
#   the ~1e-7 relative rounding of FP32 atom positions alone moves E by about
#   u * sum_i |g_i| (|x_i - t| + 1 A) -> X_TOL * that sum.
E_ABS_TOL = 1e-6
X_TOL = 16 * 2.0 ** -24


def e_relerr(e_gpu, e_ref):
    e_gpu = np.asarray(e_gpu, np.float64)
    e_ref = np.asarray(e_ref, np.float64)
    return np.abs(e_gpu - e_ref) / np.maximum(np.abs(e_ref), 1.0)


def e_ok(e_gpu, ref, genotypes):
    """Per individual: within E_TOL of max(|E|, 1), or within the FP32
    conditioning bounds above. Returns (ok, cond) where cond marks
    individuals that passed only by a conditioning bound."""
    err = np.abs(np.asarray(e_gpu, np.float64) - ref.energy)
    rel_ok = err <= E_TOL * np.maximum(np.abs(ref.energy), 1.0)
    t = np.asarray(genotypes, np.float64)[:, None, 0:3]
    sx = np.sum(np.linalg.norm(ref.atom_grad, axis=-1) * (np.linalg.norm(ref.x - t, axis=-1) + 1.0),
                axis=1)
    cond_ok = (err <= E_ABS_TOL * ref.e_abs) | (err <= X_TOL * sx)
    return rel_ok | cond_ok, (~rel_ok) & cond_ok


def g_relerr(g_gpu, g_ref):
    g_gpu = np.asarray(g_gpu, np.float64)
    g_ref = np.asarray(g_ref, np.float64)
    return np.linalg.norm(g_gpu - g_ref, axis=-1) / np.maximum(np.linalg.norm(g_ref, axis=-1), 1.0)


def near_discontinuity(prep, grd, x, tol_u=5e-5, tol_cap=1e-4):
    """Individuals whose pose sits within rounding reach of a kink of the score.

    The score is only piecewise smooth: trilinear cells change at grid
    faces, the box clamp switches at the box faces, and the 12-6/12-10 term
    switches to its cap. An FP32 and an FP64 evaluation of the same genotype
    may land on different sides of such a kink and then legitimately differ
    in the gradient (and slightly in E). Returns a boolean mask [n].
    """
    from oracle import dock_ref as R
    nx, ny, nz = grd.dims
    dims = np.array([nx, ny, nz], dtype=np.float64)
    lo = np.asarray(grd.origin, np.float64)
    hi = lo + (dims - 1) * grd.spacing
    u = (np.clip(x, lo, hi) - lo) / grd.spacing
    frac = np.abs(u - np.round(u))
    face = np.any(frac < tol_u, axis=(1, 2))
    boxf = np.any(np.abs(x - lo) < tol_u * grd.spacing, axis=(1, 2)) | \
        np.any(np.abs(x - hi) < tol_u * grd.spacing, axis=(1, 2))
    i, j = prep.pairs[:, 0], prep.pairs[:, 1]
    d = x[:, j] - x[:, i]
    r2 = np.sum(d * d, axis=-1)
    r2c = np.maximum(r2, R.R2_MIN)
    s = prep.r0 / np.sqrt(r2c)
    s6 = s ** 6
    elj = np.where(prep.pair_hb, prep.eps * (5 * s6 * s6 - 6 * s6 * s * s * s * s),
                   prep.eps * (s6 * s6 - 2 * s6))
    cap = np.any(np.abs(elj - R.E_CAP) < tol_cap * R.E_CAP, axis=1)
    clamp = np.any(np.abs(r2 - R.R2_MIN) < 1e-3 * R.R2_MIN, axis=1)
    return face | boxf | cap | clamp
