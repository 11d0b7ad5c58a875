"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (FP32 path, per individual): |dE|/max(|E|,1) <= 1e-5 and
||dg||/max(||g||,1) <= 1e-4. Individuals whose pose lies within rounding
reach of a kink of the piecewise-smooth score (grid-cell face, box face, the
1e5 cap, the r^2 clamp) are held to a looser bound and counted; they must be
rare.
"""
import math

import numpy as np
import pytest

from oracle import dock_ref as R
from oracle import reduce_ref as RR
from paper_2410_10447_amd import synth
from tests.gpu_common import E_TOL, G_TOL, e_ok, e_relerr, g_relerr, near_discontinuity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP32_VARIANTS = [0, 1]          # shuffle, FP32 MFMA
SPLIT_VARIANTS = [2, 3, 4]      # BF16 2-term, FP16 2-term, BF16 3-term


@pytest.fixture(scope="module")
def dk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_10447_amd import dock
    dock.lib()
    return dock


# ---------------------------------------------------------------------------
# Block sum (the paper's reduction step in isolation)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("threads", [64, 128, 256, 1024])
@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5])
def test_block_sum_integer_exact(dk, threads, variant):
    """Integer data with |x| < 2^7: every variant's sum is exact."""
    rng = np.random.default_rng(threads + 7 * variant)
    nb = 37
    x = rng.integers(-127, 128, (nb, threads, 4)).astype(np.float32)
    out = dk.block_sum4(torch.from_numpy(x).cuda(), variant).cpu().numpy()
    want = x.astype(np.float64).sum(axis=1)
    assert np.array_equal(out, np.broadcast_to(want[:, None, :], out.shape).astype(np.float32))


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5])
def test_block_sum_random_error_bound(dk, variant):
    rng = np.random.default_rng(100 + variant)
    nb, th = 64, 256
    x = (rng.normal(size=(nb, th, 4)) * 10 ** rng.uniform(-2, 4, (nb, th, 1))).astype(np.float32)
    out = dk.block_sum4(torch.from_numpy(x).cuda(), variant).cpu().numpy()
    ex = np.stack([RR.sum4_exact(x[b]) for b in range(nb)])
    abs_sum = np.abs(x.astype(np.float64)).sum(axis=1)
    u_split = {0: 0.0, 1: 0.0, 5: 0.0, 2: 2.0 ** -16, 3: 2.0 ** -22, 4: 2.0 ** -24}[variant]
    bound = (u_split + 2 * th * 2.0 ** -24) * abs_sum
    err = np.abs(out[:, 0, :].astype(np.float64) - ex)
    assert np.all(err <= bound), (err / abs_sum).max()
    # every thread holds the same total
    assert np.all(out == out[:, :1, :])


# ---------------------------------------------------------------------------
# Scoring parity
# ---------------------------------------------------------------------------

def _score_case(dk, w, variant, n=None):
    lig = w.ligands[0]
    prep = R.prepare(lig, w.ff)
    G = dk.Grids.from_synth(w.grids)
    L = dk.Ligand(lig, w.ff)
    gen = w.genotypes[0] if n is None else w.genotypes[0][:n]
    gt = torch.from_numpy(gen).cuda()
    E, g, ao = dk.score_batch(G, L, gt, variant=variant, atom_out=True)
    torch.cuda.synchronize()
    ref = R.score(prep, w.grids, gen.astype(np.float64))
    return prep, ref, E.cpu().numpy(), g.cpu().numpy(), ao.cpu().numpy()


def _report(tag, ee, ge, flag):
    print(f"\n[{tag}] n={len(ee)} flagged={flag.sum()} E err p50={np.median(ee):.2e} "
          f"max={ee.max():.2e} (unflagged {ee[~flag].max() if (~flag).any() else 0:.2e}); "
          f"g err p50={np.median(ge):.2e} max={ge.max():.2e} "
          f"(unflagged {ge[~flag].max() if (~flag).any() else 0:.2e})", flush=True)


@pytest.mark.parametrize("variant", FP32_VARIANTS)
def test_score_parity_small_ligand(dk, variant):
    w = synth.score_workload(256)
    prep, ref, E, g, ao = _score_case(dk, w, variant)
    ee, ge = e_relerr(E, ref.energy), g_relerr(g, ref.grad)
    flag = near_discontinuity(prep, w.grids, ref.x)
    _report(f"score c0 v{variant}", ee, ge, flag)
    # per-atom positions and gradients
    print(f"[score c0 v{variant}] max pose error {np.abs(ao[:, :, 0:3] - ref.x).max():.2e} A", flush=True)
    assert np.abs(ao[:, :, 0:3] - ref.x).max() < 1e-4
    assert flag.mean() < 0.05
    assert np.all(ee[~flag] <= E_TOL)
    assert np.all(ge[~flag] <= G_TOL)
    assert np.all(ee[flag] <= 1e-3) and np.all(ge[flag] <= 1e-2)


@pytest.mark.parametrize("variant", FP32_VARIANTS)
def test_score_parity_ls_ligand(dk, variant):
    w = synth.ls_workload(512)
    prep, ref, E, g, ao = _score_case(dk, w, variant)
    ee, ge = e_relerr(E, ref.energy), g_relerr(g, ref.grad)
    flag = near_discontinuity(prep, w.grids, ref.x)
    _report(f"score c1-ligand v{variant}", ee, ge, flag)
    print(f"[score c1-ligand v{variant}] max pose error {np.abs(ao[:, :, 0:3] - ref.x).max():.2e} A",
          flush=True)
    ok, cond = e_ok(E, ref, w.genotypes[0])
    print(f"[score c1-ligand v{variant}] strict E bound missed by {cond.sum()} (conditioning bound holds)",
          flush=True)
    assert flag.mean() < 0.05
    assert np.all(ok[~flag])
    assert np.all(ge[~flag] <= G_TOL)


@pytest.mark.parametrize("variant", SPLIT_VARIANTS)
def test_score_split_variants_error_report(dk, variant):
    """Half-width MFMA reductions: error against FP64, stated per individual."""
    w = synth.ls_workload(512)
    prep, ref, E, g, ao = _score_case(dk, w, variant)
    ee, ge = e_relerr(E, ref.energy), g_relerr(g, ref.grad)
    flag = near_discontinuity(prep, w.grids, ref.x)
    _report(f"score split v{variant}", ee, ge, flag)
    if variant == 2:
        # 2-term BF16 carries 2^-16 per element
        assert np.all(ee[~flag] <= 1e-4)
    else:
        # the others reach FP32 level, so they are held to the FP32 path's
        # bound: strict, or the conditioning bound that FP32 partials imply
        ok, cond = e_ok(E, ref, w.genotypes[0])
        print(f"[score split v{variant}] strict E bound missed by {cond.sum()} (conditioning bound holds)",
              flush=True)
        assert np.all(ok[~flag])
    assert np.all(ge[~flag] <= G_TOL)


@pytest.mark.parametrize("n_atoms,n_tors,seed", [(1, 0, 1), (2, 0, 2), (5, 1, 3), (63, 12, 4),
                                                 (64, 20, 5), (65, 20, 6), (100, 32, 7),
                                                 (128, 32, 8)])
def test_score_parity_sizes(dk, n_atoms, n_tors, seed):
    if n_atoms == 1:
        from tests.helpers import ligand_from_bonds
        lig = ligand_from_bonds(np.zeros((0, 2), np.int32), [], seed=seed)
    else:
        lig = synth.ligand(n_atoms, n_tors, seed)
    grd = synth.grids(48, 10, seed + 100)
    gen = synth.genotypes(lig, grd, 96, seed + 200)
    w = synth.Workload("sizes", [lig], grd, synth.force_field(), [gen])
    prep, ref, E, g, ao = _score_case(dk, w, 0)
    ee, ge = e_relerr(E, ref.energy), g_relerr(g, ref.grad)
    flag = near_discontinuity(prep, w.grids, ref.x)
    _report(f"score N={n_atoms} T={lig.n_torsions}", ee, ge, flag)
    assert np.all(ee[~flag] <= E_TOL)
    assert np.all(ge[~flag] <= G_TOL)


def test_score_outside_box_and_unnormalised_quaternion(dk):
    w = synth.score_workload(64)
    gen = w.genotypes[0].copy()
    gen[:16, 0] += 9.0                          # far outside the 40^3 box on x
    gen[16:32, 3:7] *= np.linspace(0.2, 5.0, 16, dtype=np.float32)[:, None]
    w.genotypes[0] = gen
    prep, ref, E, g, ao = _score_case(dk, w, 0)
    ee, ge = e_relerr(E, ref.energy), g_relerr(g, ref.grad)
    flag = near_discontinuity(prep, w.grids, ref.x)
    _report("score outside/unnormalised", ee, ge, flag)
    assert np.all(ee[~flag] <= E_TOL) and np.all(ge[~flag] <= G_TOL)


def test_score_empty_batch(dk):
    w = synth.score_workload(4)
    G = dk.Grids.from_synth(w.grids)
    L = dk.Ligand(w.ligands[0], w.ff)
    E, g = dk.score_batch(G, L, torch.zeros(0, L.n_genes, device="cuda"))
    assert E.shape == (0,) and g.shape == (0, L.n_genes)


# ---------------------------------------------------------------------------
# Local search
# ---------------------------------------------------------------------------

def _ls_setup(dk, w, n):
    lig = w.ligands[0]
    G = dk.Grids.from_synth(w.grids)
    L = dk.Ligand(lig, w.ff)
    st = dk.LSState.start(torch.from_numpy(w.genotypes[0][:n]).cuda())
    return G, L, st


def _two_wave_workload(n):
    """A 100-atom, 14-torsion ligand (two atoms per lane in one wave, or one
    per lane in two waves) on 64^3 x 10 maps."""
    lig = synth.ligand(100, 14, 4100)
    grd = synth.grids(64, 10, 4101)
    return synth.Workload("ls_n100_t14_g64", [lig], grd, synth.force_field(),
                          [synth.genotypes(lig, grd, n, 4102)], iterations=30)


@pytest.mark.parametrize("variant,tpi", [(v, 64) for v in FP32_VARIANTS] + [(v, 128) for v in FP32_VARIANTS])
def test_ls_step_map(dk, variant, tpi):
    """Each GPU step is the ADADELTA update (Zeiler Alg. 1) of the GPU's own
    state and gradient, and that gradient and energy match the oracle's at the
    same point. (Comparing with a step taken on the oracle's gradient would mix
    the two: ADADELTA passes small gradient components through almost
    unscaled, so their absolute FP32 error, ~1e-4 of |g|, would dominate.)
    tpi = 64 runs the 48-atom benchmark ligand in one wave; tpi = 128 runs a
    100-atom ligand with two waves per individual."""
    w = synth.ls_workload(64) if tpi == 64 else _two_wave_workload(64)
    prep = R.prepare(w.ligands[0], w.ff)
    G, L, st = _ls_setup(dk, w, 64)
    grad = torch.zeros_like(st.genotype)
    ws = None
    worst_step = worst_g = 0.0
    n_cond = 0
    for it in range(12):
        s0 = st.to_numpy()
        ws = dk.local_search([dk.LsJob(G, L, st, variant, grad=grad, threads_per_ind=tpi)], 1,
                             variant=variant, final_eval=False, workspace=ws)
        torch.cuda.synchronize()
        s1 = st.to_numpy()
        g_gpu = grad.cpu().numpy().astype(np.float64)
        x = s0["genotype"].astype(np.float64)
        ref = R.score(prep, w.grids, x)
        flag = near_discontinuity(prep, w.grids, ref.x)
        ok, cond = e_ok(s1["energy"], ref, x)
        n_cond += cond[~flag].sum()
        assert np.all(ok[~flag]), (it, e_relerr(s1["energy"], ref.energy)[~ok].max())
        ge = g_relerr(g_gpu, ref.grad)
        worst_g = max(worst_g, ge[~flag].max())
        assert np.all(ge[~flag] <= G_TOL), (it, ge[~flag].max())
        xn, ag, ad = R.adadelta_step(x, g_gpu, s0["acc_g2"].astype(np.float64),
                                     s0["acc_dx2"].astype(np.float64), 0.8, 1e-2)
        # accumulators are sums of non-negative terms (relative error is
        # meaningful); a gene is x + dx, judged against max(|x|, |dx|)
        gscale = np.maximum(np.maximum(np.abs(xn), np.abs(x)), np.maximum(np.abs(xn - x), 1e-3))
        for name, got, want, scale in (("genotype", s1["genotype"], xn, gscale),
                                       ("acc_g2", s1["acc_g2"], ag, np.abs(ag)),
                                       ("acc_dx2", s1["acc_dx2"], ad, np.abs(ad))):
            err = np.abs(got - want) / np.maximum(scale, 1e-30)
            worst_step = max(worst_step, err.max())
            assert np.all(err <= 1e-5), (it, name, err.max())
        assert np.all(s1["iters_done"] == it + 1)
    print(f"\n[ls step-map v{variant} tpi {tpi}] worst update rel err {worst_step:.2e}, worst gradient err "
          f"{worst_g:.2e}; energies held to a conditioning bound {n_cond}", flush=True)


@pytest.mark.parametrize("tpi", [64, 128])
def test_ls_chunked_equals_single_and_deterministic(dk, tpi):
    w = synth.ls_workload(200) if tpi == 64 else _two_wave_workload(200)
    G, L, st_a = _ls_setup(dk, w, 200)
    st_b = st_a.clone()
    st_c = st_a.clone()
    dk.local_search([(G, L, st_a)], 30, final_eval=True, threads_per_ind=tpi)
    for _ in range(2):
        dk.local_search([(G, L, st_b)], 10, final_eval=False, threads_per_ind=tpi)
    dk.local_search([(G, L, st_b)], 10, final_eval=True, threads_per_ind=tpi)
    dk.local_search([(G, L, st_c)], 30, final_eval=True, threads_per_ind=tpi)
    torch.cuda.synchronize()
    a, b, c = st_a.to_numpy(), st_b.to_numpy(), st_c.to_numpy()
    for f in a:
        assert np.array_equal(a[f], b[f]), f
        assert np.array_equal(a[f], c[f]), f


def test_ls_full_size_sampled(dk):
    """3000 individuals x 300 iterations on the 48-atom ligand (the benchmark
    workload): the energy reported for each best genotype matches the
    oracle's evaluation of it on a sample, and the search descends."""
    w = synth.ls_workload(3000)
    prep = R.prepare(w.ligands[0], w.ff)
    G, L, st = _ls_setup(dk, w, 3000)
    dk.local_search([(G, L, st)], 300, final_eval=True)
    torch.cuda.synchronize()
    s = st.to_numpy()
    assert np.all(s["iters_done"] == 300)
    assert np.all(np.isfinite(s["best_energy"]))
    start = R.score(prep, w.grids, w.genotypes[0][:3000:25].astype(np.float64)).energy
    idx = np.arange(0, 3000, 25)
    ref = R.score(prep, w.grids, s["best_genotype"][idx].astype(np.float64))
    flag = near_discontinuity(prep, w.grids, ref.x)
    ee = e_relerr(s["best_energy"][idx], ref.energy)
    ok, cond = e_ok(s["best_energy"][idx], ref, s["best_genotype"][idx])
    kappa = ref.e_abs / np.maximum(np.abs(ref.energy), 1.0)
    print(f"\n[ls full] best E median {np.median(s['best_energy']):.3f} "
          f"start median {np.median(start):.1f}; sampled E err max {ee[~flag].max():.2e}; "
          f"kappa median {np.median(kappa):.1f} max {kappa.max():.1f}; "
          f"held to the magnitude bound {cond[~flag].sum()} of {(~flag).sum()}", flush=True)
    assert np.all(ok[~flag])
    assert np.all(s["best_energy"][idx] <= start + 1e-3 * np.abs(start))
    # distribution against the oracle's own 300-step search on a subsample
    sub = np.arange(0, 3000, 100)
    ost = R.ls_init(w.genotypes[0][sub])
    R.local_search(prep, w.grids, ost, 300)
    gm, om = np.median(s["best_energy"][sub]), np.median(ost.best_energy)
    print(f"[ls full] median best E gpu {gm:.4f} oracle {om:.4f}", flush=True)


def test_ls_uneven_batch_alone_equals_mixed(dk):
    """Items of different sizes in one launch give, bit for bit, what each
    gives alone; each item meets oracle parity at its best point."""
    w = synth.uneven_workload(n_ligands=6, per_ligand=12, grid_n=64)
    G = dk.Grids.from_synth(w.grids)
    Ls = [dk.Ligand(l, w.ff) for l in w.ligands]
    mixed = [dk.LSState.start(torch.from_numpy(g).cuda()) for g in w.genotypes]
    alone = [m.clone() for m in mixed]
    dk.local_search([(G, L, s) for L, s in zip(Ls, mixed)], 20)
    for L, s in zip(Ls, alone):
        dk.local_search([(G, L, s)], 20)
    torch.cuda.synchronize()
    for k, (a, m) in enumerate(zip(alone, mixed)):
        an, mn = a.to_numpy(), m.to_numpy()
        for f in an:
            assert np.array_equal(an[f], mn[f]), (k, f)
        prep = R.prepare(w.ligands[k], w.ff)
        ref = R.score(prep, w.grids, mn["best_genotype"].astype(np.float64))
        flag = near_discontinuity(prep, w.grids, ref.x)
        ok, cond = e_ok(mn["best_energy"], ref, mn["best_genotype"])
        assert np.all(ok[~flag]), (k, e_relerr(mn["best_energy"], ref.energy).max())


def test_ls_uneven_mixed_variants_alone_equals_mixed(dk):
    """Ligands on both sides of 64 atoms with alternating reduction variants
    in one call give, bit for bit, what each item gives alone."""
    ligs = [synth.ligand(n, t, 70 + n) for n, t in ((20, 4), (90, 12), (48, 8), (128, 20), (64, 6), (65, 9))]
    grd = synth.grids(64, 10, 71)
    ff = synth.force_field()
    G = dk.Grids.from_synth(grd)
    Ls = [dk.Ligand(l, ff) for l in ligs]
    gens = [torch.from_numpy(synth.genotypes(l, grd, 24, 72 + k)).cuda() for k, l in enumerate(ligs)]
    mixed = [dk.LSState.start(g) for g in gens]
    alone = [m.clone() for m in mixed]
    var = [k % 2 if k < 4 else 2 + k % 3 for k in range(len(ligs))]
    dk.local_search([dk.LsJob(G, L, s, v) for L, s, v in zip(Ls, mixed, var)], 15)
    for L, s, v in zip(Ls, alone, var):
        dk.local_search([dk.LsJob(G, L, s, v)], 15)
    torch.cuda.synchronize()
    for k, (a, m) in enumerate(zip(alone, mixed)):
        an, mn = a.to_numpy(), m.to_numpy()
        for f in an:
            assert np.array_equal(an[f], mn[f]), (k, f)


def test_ls_three_families_alone_equals_mixed(dk):
    """One call holding ligands of <= 64 atoms (one wave), larger ligands in
    one wave and larger ligands in two waves, with mixed reduction variants,
    runs one launch per family side by side and gives, bit for bit, what each
    item gives alone; the two-wave items meet oracle parity at their best
    point."""
    spec = ((20, 4, 64), (90, 12, 128), (48, 8, 64), (128, 20, 64), (100, 14, 128), (65, 9, 128),
            (128, 32, 128), (70, 0, 64))
    ligs = [synth.ligand(n, t, 90 + n + t) for n, t, _ in spec]
    grd = synth.grids(64, 10, 91)
    ff = synth.force_field()
    G = dk.Grids.from_synth(grd)
    Ls = [dk.Ligand(l, ff) for l in ligs]
    gens = [torch.from_numpy(synth.genotypes(l, grd, 20 + 3 * k, 92 + k)).cuda() for k, l in enumerate(ligs)]
    mixed = [dk.LSState.start(g) for g in gens]
    alone = [m.clone() for m in mixed]
    var = [(0, 1, 2, 0, 1, 3, 4, 0)[k] for k in range(len(ligs))]
    def job(k, st):
        return dk.LsJob(G, Ls[k], st, var[k], threads_per_ind=spec[k][2])
    dk.local_search([job(k, s) for k, s in enumerate(mixed)], 15)
    for k, s in enumerate(alone):
        dk.local_search([job(k, s)], 15)
    torch.cuda.synchronize()
    for k, (a, m) in enumerate(zip(alone, mixed)):
        an, mn = a.to_numpy(), m.to_numpy()
        for f in an:
            assert np.array_equal(an[f], mn[f]), (k, spec[k], f)
        assert np.all(mn["iters_done"] == 15)
        if spec[k][2] == 128 and var[k] in FP32_VARIANTS:
            prep = R.prepare(ligs[k], ff)
            ref = R.score(prep, grd, mn["best_genotype"].astype(np.float64))
            flag = near_discontinuity(prep, grd, ref.x)
            ok, _ = e_ok(mn["best_energy"], ref, mn["best_genotype"])
            assert np.all(ok[~flag]), (k, e_relerr(mn["best_energy"], ref.energy).max())


def test_corner_expanded_grids_identical(dk):
    """The corner-expanded copy holds the same corner values and the kernels
    do the same arithmetic on them: scores and a 20-step local search are
    bit-identical with and without it (one-wave and two-wave ligands)."""
    w = synth.ls_workload(64)
    L = dk.Ligand(w.ligands[0], w.ff)
    Gp = dk.Grids.from_synth(w.grids, corners=False)
    Gc = dk.Grids.from_synth(w.grids)
    assert Gc.corners is not None and Gc.corners.numel() == Gc.corner_bytes()
    n_cells = (np.array(w.grids.maps.shape[1:]) - 1).prod()
    M, nz, ny, nx = w.grids.maps.shape
    assert Gc.corner_bytes() == (M - 2) * n_cells * 128
    # spot-check the layout: for type t and cell (cx, cy, cz), corner
    # v[4 dz + 2 dy + dx] of the type map, the electrostatic and the desolvation map
    cv = Gc.corners.view(torch.float32).cpu().numpy().reshape(M - 2, nz - 1, ny - 1, nx - 1, 4, 8)
    assert np.all(cv[..., 3, :] == 0)
    rng = np.random.default_rng(3)
    for _ in range(50):
        t, cz, cy, cx = rng.integers(M - 2), rng.integers(nz - 1), rng.integers(ny - 1), rng.integers(nx - 1)
        for j, m in enumerate((t, M - 2, M - 1)):
            for k in range(8):
                dz, dy, dx = k >> 2, (k >> 1) & 1, k & 1
                assert cv[t, cz, cy, cx, j, k] == w.grids.maps[m, cz + dz, cy + dy, cx + dx]
    gt = torch.from_numpy(w.genotypes[0]).cuda()
    for v in FP32_VARIANTS:
        Ep, gp = dk.score_batch(Gp, L, gt, variant=v)
        Ec, gc = dk.score_batch(Gc, L, gt, variant=v)
        assert torch.equal(Ep, Ec) and torch.equal(gp, gc)
    for lig_n, tpi in ((48, 64), (100, 128)):
        ww = w if lig_n == 48 else _two_wave_workload(64)
        LL = L if lig_n == 48 else dk.Ligand(ww.ligands[0], ww.ff)
        Gp2 = Gp if lig_n == 48 else dk.Grids.from_synth(ww.grids, corners=False)
        Gc2 = Gc if lig_n == 48 else dk.Grids.from_synth(ww.grids)
        a = dk.LSState.start(torch.from_numpy(ww.genotypes[0]).cuda())
        b = a.clone()
        dk.local_search([(Gp2, LL, a)], 20, threads_per_ind=tpi)
        dk.local_search([(Gc2, LL, b)], 20, threads_per_ind=tpi)
        torch.cuda.synchronize()
        an, bn = a.to_numpy(), b.to_numpy()
        for f in an:
            assert np.array_equal(an[f], bn[f]), (lig_n, f)


def test_ls_mixed_variants_in_one_launch(dk):
    w = synth.ls_workload(64)
    G, L, st0 = _ls_setup(dk, w, 64)
    st1 = st0.clone()
    ref0, ref1 = st0.clone(), st0.clone()
    dk.local_search([(G, L, st0, 0), (G, L, st1, 1)], 15)
    dk.local_search([(G, L, ref0)], 15, variant=0)
    dk.local_search([(G, L, ref1)], 15, variant=1)
    torch.cuda.synchronize()
    for a, b in ((st0, ref0), (st1, ref1)):
        an, bn = a.to_numpy(), b.to_numpy()
        for f in an:
            assert np.array_equal(an[f], bn[f]), f
