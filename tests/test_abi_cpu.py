"""C-ABI checks that need no GPU: exported symbols, host-side ligand
preparation (bit-exact against the oracle's independent BFS construction),
and argument validation of every entry point (errors are returned before any
device work, so these run on a machine without a GPU)."""
import ctypes as C
import re

import numpy as np
import pytest

from oracle import dock_ref as R
from paper_2410_10447_amd import dock, synth
from tests.helpers import ligand_from_bonds, load_golden

FF = synth.force_field()


def test_library_exports_every_declared_symbol():
    L = dock.lib()
    hdr = open(__import__("os").path.join(dock.__file__.rsplit("/", 2)[0], "include", "dock.h")).read()
    declared = set(re.findall(r"^\s*(?:int32_t|const char\*)\s+(dock_\w+)\s*\(", hdr, re.M))
    assert declared == set(dock.ABI_SYMBOLS)
    for name in declared:
        assert hasattr(L, name)
    assert L.dock_abi_version() == dock.ABI_VERSION == 11


def _check_prep(lig):
    h = dock.Ligand(lig, FF, upload=False)
    ex = h.export()
    p = R.prepare(lig, FF)
    N, T = lig.n_atoms, lig.n_torsions
    assert (h.n_atoms, h.n_torsions, h.n_genes, h.n_pairs) == (N, T, 7 + T, len(p.pairs))
    assert h.n_fragments == p.n_frag
    # depth-first order: a permutation, root first, every subtree contiguous
    order = ex["order"]
    assert sorted(order.tolist()) == list(range(N)) and order[0] == 0
    # torsions: same axis atoms; moving range = the oracle's BFS moving set
    for k in range(T):
        a, b, first, end = ex["torsions"][k]
        assert (a, b) == tuple(p.axis[k])
        assert set(order[first:end].tolist()) == set(np.nonzero(p.moving[k])[0].tolist())
        assert order[first] == b
    # fragments: same partition
    part_c = {}
    part_o = {}
    for i in range(N):
        part_c.setdefault(int(ex["fragment"][i]), set()).add(i)
        part_o.setdefault(int(p.frag[i]), set()).add(i)
    assert sorted(map(sorted, part_c.values())) == sorted(map(sorted, part_o.values()))
    # pair list and hydrogen-bond flags, decoded from the kernel's batches
    assert np.array_equal(ex["pairs"], p.pairs)
    assert np.array_equal(ex["pair_hb"], p.pair_hb)
    _check_batches(ex["batches"], h.n_copies, N, p, order)
    # the depth-first order is the one defined by the header: neighbours in
    # increasing index, each atom at its first visit (independent recursive
    # construction)
    adj = {i: [] for i in range(N)}
    for u, v in lig.bonds:
        adj[int(u)].append(int(v)); adj[int(v)].append(int(u))
    want = []
    seen = set()

    def visit(u):
        seen.add(u)
        want.append(u)
        for v in sorted(adj[u]):
            if v not in seen:
                visit(v)
    visit(0)
    assert order.tolist() == want


def _check_batches(b, C, N, p, order):
    """Batch records: valid pairs are the pair list; every lane of a batch,
    unused lanes included, owns two (copy, atom) slots no other lane of the
    batch touches; unused lanes take free copies of real atoms, or slots of
    the "atoms" N .. S-1 (S the power-of-two stride >= max(N, 16)) that are
    never summed; C * S fits the accumulator."""
    S = max(16, 1 << (N - 1).bit_length())
    cap = 320 if N <= 64 else 384
    assert C * S <= cap and 2 <= C <= 15
    got = []
    for row in b:
        slots = []
        for r in row.tolist():
            i, j = r & 127, (r >> 7) & 127
            ci, cj = (r >> 14) & 15, (r >> 18) & 15
            if not (r >> 31) & 1:
                assert (r >> 22) == 0, "unused lane with flags"
                for c, a in ((ci, i), (cj, j)):
                    assert c < C and a < S, (c, a)
                slots += [(ci, i), (cj, j)]
                continue
            assert i < N and j < N and ci < C and cj < C
            slots += [(ci, i), (cj, j)]
            a, bb = int(order[i]), int(order[j])
            got.append((min(a, bb), max(a, bb), (r >> 22) & 1))
        assert len(slots) == len(set(slots)) == 128
    got.sort()
    want = sorted((int(a), int(bb), int(hb)) for (a, bb), hb in zip(p.pairs, p.pair_hb))
    assert got == want
    # the batch count stays at the lower bound max(P/64, max degree / C)
    P = len(p.pairs)
    if P:
        deg = np.bincount(p.pairs.ravel(), minlength=N)
        lb = max(-(-P // 64), -(-int(deg.max()) // C))
        assert len(b) <= lb + 1, (len(b), lb)


@pytest.mark.parametrize("wl", ["score", "ls"])
def test_prep_bitexact_named_workloads(wl):
    w = synth.score_workload(1) if wl == "score" else synth.ls_workload(1)
    _check_prep(w.ligands[0])


def test_prep_bitexact_uneven_batch_ligands():
    w = synth.uneven_workload(n_ligands=64, per_ligand=1, grid_n=8)
    for lig in w.ligands:
        _check_prep(lig)


@pytest.mark.parametrize("name", ["prep_chain7.json", "prep_branched9.json", "prep_rigid6.json"])
def test_prep_golden(name):
    g = load_golden(name)
    lig = ligand_from_bonds(g["bonds"], g["rot_bonds"])
    _check_prep(lig)
    ex = dock.Ligand(lig, FF, upload=False).export()
    assert ex["pairs"].tolist() == g["pairs"]


@pytest.mark.parametrize("n,t,seed", [(1, 0, 3), (2, 0, 4), (3, 0, 5), (4, 1, 6), (64, 20, 7),
                                      (65, 20, 8), (127, 32, 9), (128, 32, 10)])
def test_prep_edge_sizes(n, t, seed):
    if n == 1:
        lig = ligand_from_bonds(np.zeros((0, 2), np.int32), [])
    else:
        lig = synth.ligand(n, t, seed)
    _check_prep(lig)


def _desc_from(lig, **over):
    xyz = np.ascontiguousarray(lig.xyz, np.float64)
    chg = np.ascontiguousarray(lig.charge, np.float64)
    cls = np.ascontiguousarray(lig.cls, np.int32)
    bonds = np.ascontiguousarray(lig.bonds, np.int32)
    rot = np.ascontiguousarray(lig.rot_bonds, np.int32)
    arrs = dict(xyz=xyz, charge=chg, cls=cls, bonds=bonds, rot=rot)
    arrs.update(over)
    ffp, keep = dock.ff_params(FF)
    d = dock.LigandDesc()
    d.n_atoms = arrs.get("n_atoms", xyz.shape[0])
    d.n_torsions = arrs.get("n_torsions", arrs["rot"].shape[0])
    d.root_atom = arrs.get("root", 0)
    d.n_bonds = arrs.get("n_bonds", arrs["bonds"].shape[0])
    d.xyz = arrs["xyz"].ctypes.data_as(C.POINTER(C.c_double))
    d.charge = arrs["charge"].ctypes.data_as(C.POINTER(C.c_double))
    d.cls = arrs["cls"].ctypes.data_as(C.POINTER(C.c_int32))
    d.bonds = arrs["bonds"].ctypes.data_as(C.POINTER(C.c_int32))
    d.rot_bonds = arrs["rot"].ctypes.data_as(C.POINTER(C.c_int32))
    d.ff = C.pointer(ffp)
    return d, (arrs, ffp, keep)


def _create(d):
    h = C.c_void_p()
    st = dock.lib().dock_create_ligand(C.byref(d), C.byref(h))
    if st == 0:
        dock.lib().dock_destroy_ligand(h)
    return st


def _read_pass(lane):
    """gfx950 16-byte LDS read pass of a lane (4 passes of 16 lanes): lane bit 5
    and the parity of lane bits 2..4."""
    b = (lane >> 2) & 7
    return 2 * (lane >> 5) + ((b ^ (b >> 1) ^ (b >> 2)) & 1)


def _bank_repeats(batches, n_atoms):
    """Extra LDS passes per batch of the pair loop's accesses under the bank
    model measured on gfx950: reads conflict within a read pass when distinct
    addresses agree mod 16 (16-byte units), writes within an aligned 8-lane
    group when distinct addresses agree mod 8."""
    S = max(16, 1 << (n_atoms - 1).bit_length())
    passes = [[l for l in range(64) if _read_pass(l) == p] for p in range(4)]
    rd = wr = 0
    for row in batches.astype(np.int64):
        i, j, ci, cj = row & 127, (row >> 7) & 127, (row >> 14) & 15, (row >> 18) & 15
        for a, c in ((i, ci), (j, cj)):
            slot = (c * S + a).tolist()
            for addr in (slot, a.tolist()):
                for ln in passes:
                    q = {}
                    for l in ln:
                        q.setdefault(addr[l] % 16, set()).add(addr[l])
                    rd += max(len(v) for v in q.values()) - 1
            for w in range(8):
                q = {}
                for l in range(8 * w, 8 * w + 8):
                    q.setdefault(slot[l] % 8, set()).add(slot[l])
                wr += max(len(v) for v in q.values()) - 1
    return rd / max(len(batches), 1), wr / max(len(batches), 1)


def test_read_pass_sets():
    passes = [sorted(l for l in range(64) if _read_pass(l) == p) for p in range(4)]
    assert passes[0] == [0, 1, 2, 3, 12, 13, 14, 15, 20, 21, 22, 23, 24, 25, 26, 27]
    assert all(len(p) == 16 for p in passes)
    # every aligned 8-lane write group takes 4 lanes of each read pass of its half
    for w in range(8):
        got = sorted(_read_pass(l) for l in range(8 * w, 8 * w + 8))
        half = w // 4
        assert got == [2 * half] * 4 + [2 * half + 1] * 4


def test_lane_arrangement_spreads_banks():
    """The host arrangement keeps the pair loop's LDS repeats (reads and
    writes, per batch) below half of what the same records give on randomly
    permuted lanes, for the benchmark ligand and the uneven batch's ligands."""
    ff = synth.force_field()
    rng = np.random.default_rng(5)
    ligs = [synth.ls_workload(1).ligands[0]] + synth.uneven_workload(n_ligands=16, per_ligand=1,
                                                                     grid_n=8).ligands
    for k, lig in enumerate(ligs):
        L = dock.Ligand(lig, ff, upload=False)
        if L.n_batches == 0:
            continue
        b = L.export()["batches"]
        shuffled = np.stack([row[rng.permutation(64)] for row in b])
        rd, wr = _bank_repeats(b, L.n_atoms)
        rd0, wr0 = _bank_repeats(shuffled, L.n_atoms)
        assert rd + wr <= 0.5 * (rd0 + wr0), (L.n_atoms, rd, wr, rd0, wr0)
        if k == 0:
            # random lanes give about 47 repeats per batch for this ligand
            assert rd + wr <= 15.0, (rd, wr)


def test_create_ligand_rejects_bad_topologies():
    lig = synth.ligand(12, 3, 1)
    d, keep = _desc_from(lig)
    assert _create(d) == 0
    bad_bonds = lig.bonds.copy(); bad_bonds[3] = bad_bonds[2]          # duplicate -> not a tree
    d, keep = _desc_from(lig, bonds=bad_bonds)
    assert _create(d) == dock.DOCK_EINVAL and "bond" in dock.last_error()
    cyc = lig.bonds.copy(); cyc[5] = [0, 1] if tuple(cyc[0]) != (0, 1) else [1, 2]
    d, keep = _desc_from(lig, bonds=cyc)
    assert _create(d) == dock.DOCK_EINVAL
    # a terminal bond is not rotatable
    deg = np.bincount(lig.bonds.ravel(), minlength=12)
    term = [k for k, (u, v) in enumerate(lig.bonds) if deg[u] == 1 or deg[v] == 1][0]
    d, keep = _desc_from(lig, rot=np.array([term], np.int32))
    assert _create(d) == dock.DOCK_EINVAL and "internal" in dock.last_error()
    d, keep = _desc_from(lig, rot=np.array([lig.rot_bonds[0]] * 2, np.int32))
    assert _create(d) == dock.DOCK_EINVAL
    d, keep = _desc_from(lig, cls=np.full(12, 99, np.int32))
    assert _create(d) == dock.DOCK_EINVAL and "class" in dock.last_error()
    d, keep = _desc_from(lig, root=12)
    assert _create(d) == dock.DOCK_EINVAL
    xyz = lig.xyz.copy(); xyz[0, 0] = np.nan
    d, keep = _desc_from(lig, xyz=xyz)
    assert _create(d) == dock.DOCK_EINVAL


def test_ring_ligands_bitexact_and_ring_bonds_rejected():
    """Ligands with rings (planar rings joined by single bonds): the C++
    preparation matches the oracle's BFS construction; a rotatable bond
    inside a ring, a bond count outside [N - 1, 4 N] and a disconnected
    graph are rejected."""
    for seed, (nr, nc, t) in enumerate([(1, 4, 2), (2, 6, 4), (3, 10, 8), (4, 20, 12), (6, 30, 20),
                                        (1, 0, 0), (2, 0, 1), (8, 40, 32)]):
        lig = synth.ring_ligand(nr, nc, t, 700 + seed)
        assert lig.bonds.shape[0] == lig.n_atoms - 1 + nr
        _check_prep(lig)
    lig = synth.ring_ligand(2, 6, 3, 720)
    ring_bond = lig.n_atoms - 1 + 1      # some bond of a ring: every bond not listed as single
    single = set()
    for k in lig.rot_bonds.tolist():
        single.add(k)
    deg = np.bincount(lig.bonds.ravel(), minlength=lig.n_atoms)
    in_ring = []
    for k, (u, v) in enumerate(lig.bonds):
        # a bond is in a ring iff removing it leaves the graph connected
        rest = np.delete(lig.bonds, k, axis=0)
        adj = {i: [] for i in range(lig.n_atoms)}
        for a, b in rest:
            adj[int(a)].append(int(b)); adj[int(b)].append(int(a))
        seen, stack = {0}, [0]
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if y not in seen:
                    seen.add(y); stack.append(y)
        if len(seen) == lig.n_atoms and deg[u] >= 2 and deg[v] >= 2:
            in_ring.append(k)
    assert in_ring and ring_bond >= 0
    d, keep = _desc_from(lig, rot=np.array([in_ring[0]], np.int32))
    assert _create(d) == dock.DOCK_EINVAL and "ring" in dock.last_error()
    with pytest.raises(ValueError):
        R.prepare(synth.Ligand(xyz=lig.xyz, charge=lig.charge, cls=lig.cls, bonds=lig.bonds,
                               rot_bonds=np.array([in_ring[0]], np.int32)), FF)
    d, keep = _desc_from(lig, n_bonds=lig.n_atoms - 2)
    assert _create(d) == dock.DOCK_EINVAL and "n_bonds" in dock.last_error()
    d, keep = _desc_from(lig, n_bonds=4 * lig.n_atoms + 1)
    assert _create(d) == dock.DOCK_EINVAL
    # two rings side by side, not joined: not connected
    a = synth.ring_ligand(1, 0, 0, 721)
    bonds = np.concatenate([a.bonds, a.bonds + 6, np.array([[0, 3]], np.int32)])
    xyz = np.concatenate([a.xyz, a.xyz + 10.0])
    d, keep = _desc_from(a, bonds=bonds, xyz=xyz, charge=np.zeros(12), cls=np.zeros(12, np.int32), n_atoms=12,
                         rot=np.zeros(0, np.int32))
    assert _create(d) == dock.DOCK_EINVAL and "connect" in dock.last_error()


def test_create_ligand_limits():
    big = synth.ligand(129, 3, 2)
    d, keep = _desc_from(big)
    assert _create(d) == dock.DOCK_EUNSUPPORTED
    lig = synth.ligand(60, 40, 3)   # 33+ torsions requested; generator caps to internal bonds
    if lig.n_torsions > 32:
        d, keep = _desc_from(lig)
        assert _create(d) == dock.DOCK_EUNSUPPORTED
    d, keep = _desc_from(synth.ligand(5, 1, 4), n_atoms=0)
    assert _create(d) == dock.DOCK_EINVAL


def test_batch_calls_validate_before_device_work():
    L = dock.lib()
    vp = C.c_void_p
    assert L.dock_score_batch(None, None, 1, None, None, None, None, None) == dock.DOCK_EINVAL
    lig = dock.Ligand(synth.ligand(10, 2, 5), FF, upload=False)
    d = dock.GridDesc(nx=8, ny=8, nz=8, n_maps=10, spacing=0.375)
    g = C.c_void_p()
    fake = vp(0x1000)     # never dereferenced: validation fails first or no launch happens
    assert L.dock_create_grids(C.byref(d), None, C.byref(g)) == dock.DOCK_EINVAL
    d2 = dock.GridDesc(nx=1, ny=8, nz=8, n_maps=10, spacing=0.375)
    assert L.dock_create_grids(C.byref(d2), fake, C.byref(g)) == dock.DOCK_EINVAL
    d3 = dock.GridDesc(nx=8, ny=8, nz=8, n_maps=2, spacing=0.375)
    assert L.dock_create_grids(C.byref(d3), fake, C.byref(g)) == dock.DOCK_EINVAL
    d4 = dock.GridDesc(nx=8, ny=8, nz=8, n_maps=10, spacing=0.0)
    assert L.dock_create_grids(C.byref(d4), fake, C.byref(g)) == dock.DOCK_EINVAL
    assert L.dock_create_grids(C.byref(d), fake, C.byref(g)) == dock.DOCK_OK
    # corner-expanded copy: size, and validation before any launch
    nb = C.c_int64()
    assert L.dock_grids_corner_bytes(g, C.byref(nb)) == dock.DOCK_OK and nb.value == 8 * 7 * 7 * 7 * 128
    assert L.dock_grids_corner_bytes(None, C.byref(nb)) == dock.DOCK_EINVAL
    assert L.dock_grids_bind_corners(None, fake, nb.value, None) == dock.DOCK_EINVAL
    assert L.dock_grids_bind_corners(g, fake, nb.value - 1, None) == dock.DOCK_EINVAL
    assert L.dock_grids_bind_corners(g, vp(0x1008), nb.value, None) == dock.DOCK_EINVAL
    assert L.dock_grids_bind_corners(g, None, 0, None) == dock.DOCK_OK      # unbind: no device work
    # ligand never uploaded
    st = L.dock_score_batch(g, lig.handle, 4, fake, fake, fake, None, None)
    assert st == dock.DOCK_EINVAL and "uploaded" in dock.last_error()
    # a grid with too few type maps for the ligand's classes
    d5 = dock.GridDesc(nx=8, ny=8, nz=8, n_maps=3, spacing=0.375)
    g5 = C.c_void_p()
    assert L.dock_create_grids(C.byref(d5), fake, C.byref(g5)) == dock.DOCK_OK
    item = (dock.LsItem * 1)()
    item[0].grids = g.value
    item[0].ligand = lig.handle.value
    item[0].n = 4
    item[0].variant = -1
    o = dock.LsOpts(iterations=10, rho=0.8, eps=1e-2, variant=0, threads_per_ind=0, flags=1)
    # rows of another gene count than the ligand's are rejected (the kernels
    # would index them with the ligand's G)
    for bad_g in (0, lig.n_genes - 1, lig.n_genes + 1):
        item[0].n_genes = bad_g
        st = L.dock_local_search_batch(item, 1, C.byref(o), fake, 1 << 20, None)
        assert st == dock.DOCK_EINVAL and "n_genes" in dock.last_error()
    item[0].n_genes = lig.n_genes
    st = L.dock_local_search_batch(item, 1, C.byref(o), fake, 1 << 20, None)
    assert st == dock.DOCK_EINVAL and "uploaded" in dock.last_error()
    # the same check in the Solis-Wets call
    for bad_g in (lig.n_genes - 1, lig.n_genes + 1):
        so = dock.SwOpts(iterations=2, n_genes=bad_g, n_success=4, n_failure=4, variant=0)
        st = L.dock_solis_wets_batch(g, lig.handle, 4, fake, fake, fake, fake, fake, fake, fake,
                                     C.byref(so), None, None)
        assert st == dock.DOCK_EINVAL and "n_genes" in dock.last_error()
    for bad in (dict(rho=1.0), dict(rho=0.0), dict(eps=0.0), dict(iterations=-1), dict(variant=9),
                dict(flags=4), dict(threads_per_ind=96), dict(threads_per_ind=512)):
        kw = dict(iterations=10, rho=0.8, eps=1e-2, variant=0, threads_per_ind=0, flags=1)
        kw.update(bad)
        ob = dock.LsOpts(**kw)
        assert L.dock_local_search_batch(item, 1, C.byref(ob), fake, 1 << 20, None) in (
            dock.DOCK_EINVAL, dock.DOCK_EUNSUPPORTED)
    # two individuals per wave: only for ligands of <= 32 atoms and 32 genes
    big = dock.Ligand(synth.ligand(40, 3, 9), FF, upload=False)
    item2 = (dock.LsItem * 1)()
    item2[0].grids = g.value
    item2[0].ligand = big.handle.value
    item2[0].n = 4
    item2[0].n_genes = big.n_genes
    item2[0].variant = -1
    item2[0].flags = dock.ITEM_TWO_PER_WAVE
    st = L.dock_local_search_batch(item2, 1, C.byref(o), fake, 1 << 20, None)
    assert st == dock.DOCK_EUNSUPPORTED and "two individuals" in dock.last_error()
    item2[0].flags = 4
    assert L.dock_local_search_batch(item2, 1, C.byref(o), fake, 1 << 20, None) == dock.DOCK_EINVAL
    # the library-resident variant validates the same way, before any device work
    for bad_g in (lig.n_genes - 1, lig.n_genes + 1):
        item[0].n_genes = bad_g
        st = L.dock_local_search_batch_static(item, 1, C.byref(o), None)
        assert st == dock.DOCK_EINVAL and "n_genes" in dock.last_error()
    item[0].n_genes = lig.n_genes
    st = L.dock_local_search_batch_static(item, 1, C.byref(o), None)
    assert st == dock.DOCK_EINVAL and "uploaded" in dock.last_error()
    assert L.dock_local_search_batch_static(item, 1, None, None) == dock.DOCK_EINVAL
    assert L.dock_local_search_batch_static(None, 1, C.byref(o), None) == dock.DOCK_EINVAL
    many = (dock.LsItem * (dock.STATIC_MAX_ITEMS + 1))()
    st = L.dock_local_search_batch_static(many, dock.STATIC_MAX_ITEMS + 1, C.byref(o), None)
    assert st == dock.DOCK_EINVAL and "DOCK_STATIC_MAX_ITEMS" in dock.last_error()
    assert L.dock_local_search_batch_static(item, 0, C.byref(o), None) == dock.DOCK_OK   # nothing to do
    # the launch-count query validates the same way, before any device work
    nl = C.c_int32(-1)
    assert L.dock_ls_launches(item, 1, C.byref(o), None) == dock.DOCK_EINVAL
    st = L.dock_ls_launches(item, 1, C.byref(o), C.byref(nl))
    assert st == dock.DOCK_EINVAL and "uploaded" in dock.last_error()
    assert L.dock_ls_launches(item, 0, C.byref(o), C.byref(nl)) == dock.DOCK_OK and nl.value == 0
    for bad in (dict(flags=4), dict(threads_per_ind=96)):
        kw = dict(iterations=10, rho=0.8, eps=1e-2, variant=0, threads_per_ind=0, flags=1)
        kw.update(bad)
        ob = dock.LsOpts(**kw)
        assert L.dock_ls_launches(item, 1, C.byref(ob), C.byref(nl)) in (dock.DOCK_EINVAL, dock.DOCK_EUNSUPPORTED)
    b = C.c_int64()
    assert L.dock_ls_workspace_bytes(3, C.byref(b)) == 0 and b.value >= 64 + 3 * 64
    assert L.dock_ls_workspace_bytes(-1, C.byref(b)) == dock.DOCK_EINVAL
    assert L.dock_block_sum4(fake, fake, 1, 65, 0, 1, None) == dock.DOCK_EINVAL
    assert L.dock_block_sum4(fake, fake, 1, 64, 7, 1, None) == dock.DOCK_EINVAL
    assert L.dock_block_sum4(fake, fake, 1, 2048, 0, 1, None) == dock.DOCK_EINVAL
    assert L.dock_destroy_grids(g) == 0 and L.dock_destroy_grids(g5) == 0
    assert L.dock_destroy_grids(None) == 0 and L.dock_destroy_ligand(None) == 0


def test_binding_rejects_item_arrays_shorter_than_jobs():
    """A prebuilt item array must cover every job: the binding checks its
    length before the library reads it (the C ABI takes a count only)."""
    items = dock.make_items([])       # one zeroed record
    jobs = [None, None]
    with pytest.raises(ValueError, match="items shorter"):
        dock.ls_launches(jobs, 1, items=items)
    with pytest.raises(ValueError, match="items shorter"):
        dock.local_search(jobs, 1, items=items)
    with pytest.raises(ValueError, match="items shorter"):
        dock.local_search_static(jobs, 1, items=items)


def test_row_selection_calls_validate_before_device_work():
    L = dock.lib()
    vp = C.c_void_p
    fake = vp(0x1000)
    cnt = vp(0x2000)
    assert L.dock_select_rows(fake, -1, 0.5, fake, cnt, None) == dock.DOCK_EINVAL
    assert L.dock_select_rows(fake, 4, 0.5, fake, None, None) == dock.DOCK_EINVAL
    assert L.dock_select_rows(None, 4, 0.5, fake, cnt, None) == dock.DOCK_EINVAL
    assert L.dock_select_rows(fake, 4, float("nan"), fake, cnt, None) == dock.DOCK_EINVAL
    assert L.dock_select_rows(vp(0x1002), 4, 0.5, fake, cnt, None) == dock.DOCK_EINVAL
    for fn in (L.dock_gather_rows, L.dock_scatter_rows):
        assert fn(fake, 4, 0, fake, 2, fake, None) == dock.DOCK_EINVAL          # row < 1
        assert fn(fake, -1, 3, fake, 2, fake, None) == dock.DOCK_EINVAL
        assert fn(fake, 4, 3, fake, -2, fake, None) == dock.DOCK_EINVAL
        assert fn(None, 4, 3, fake, 2, fake, None) == dock.DOCK_EINVAL
        assert fn(fake, 4, 3, None, 2, fake, None) == dock.DOCK_EINVAL
        assert fn(fake, 4, 3, fake, 2, vp(0x1001), None) == dock.DOCK_EINVAL
        assert fn(fake, 1 << 30, 3, fake, 2, fake, None) == dock.DOCK_EINVAL    # > 2^31 - 1 elements
    # m == 0: nothing to do (gather: m is the fifth argument, scatter: the second)
    assert L.dock_gather_rows(None, 4, 3, None, 0, None, None) == dock.DOCK_OK
    assert L.dock_scatter_rows(None, 0, 3, None, 4, None, None) == dock.DOCK_OK


def test_ga_step_rejects_bad_descriptors_before_any_device_work():
    """Argument checks of dock_ga_step run on the host and need no GPU."""
    L = dock.lib()
    assert L.dock_ga_step(None, None) == dock.DOCK_EINVAL
    fake = 1 << 20                      # never dereferenced: every call below fails a check
    base = dict(genotypes=fake, energies=fake + 4096, candidates=fake + 8192, coins=fake + 12288,
                cuts=fake + 16384, mut_coin=fake + 20480, mut_delta=fake + 24576,
                children=fake + (1 << 16), best=fake + (1 << 17),
                n_runs=2, pop=3, n_genes=7, p_tournament=0.6, p_crossover=0.8, p_mutation=0.02,
                elitism=1)
    bad = [dict(n_runs=0), dict(pop=-1), dict(n_genes=0), dict(n_genes=40),
           dict(n_runs=1 << 16, pop=1 << 16, n_genes=2), dict(p_crossover=float("nan")),
           dict(elitism=2), dict(candidates=fake + 8200), dict(cuts=fake + 16388),
           dict(children=fake + 8), dict(best=None), dict(genotypes=None)]
    for change in bad:
        d = dock.GaStepDesc(**{**base, **change})
        assert L.dock_ga_step(C.byref(d), None) == dock.DOCK_EINVAL, change
        assert "dock_ga_step" in dock.last_error()


def test_binding_validates_state_tensors():
    """The binding rejects state, gradient, draw and scale tensors that do not
    fit the ligand (wrong gene width or length, dtype, layout or device)
    before the C call, which receives bare pointers. Checked with CPU
    tensors: the shape, dtype and layout checks come before the device one."""
    import torch
    w = synth.ls_workload(4)
    lig = dock.Ligand(w.ligands[0], w.ff, upload=False)
    G = lig.n_genes
    n = 5

    def state(**over):
        f = dict(genotype=torch.zeros(n, G), acc_g2=torch.zeros(n, G), acc_dx2=torch.zeros(n, G),
                 best_genotype=torch.zeros(n, G), best_energy=torch.zeros(n), energy=torch.zeros(n),
                 iters_done=torch.zeros(n, dtype=torch.int32))
        f.update(over)
        return dock.LSState(**f)

    grids_stub = object()          # never reached: validation fails first
    bad = [
        (dict(genotype=torch.zeros(n, G - 1)), "shape"),
        (dict(acc_g2=torch.zeros(n, G + 1)), "shape"),
        (dict(best_genotype=torch.zeros(n + 1, G)), "shape"),
        (dict(best_energy=torch.zeros(n - 1)), "shape"),
        (dict(acc_dx2=torch.zeros(n, G, dtype=torch.float64)), "float32"),
        (dict(iters_done=torch.zeros(n, dtype=torch.int64)), "int32"),
        (dict(energy=torch.zeros(2 * n)[::2]), "contiguous"),
        (dict(genotype=torch.zeros(G, n).t()), "contiguous"),
        ({}, "CUDA"),
    ]
    for over, what in bad:
        with pytest.raises(ValueError, match=what):
            dock.make_items([dock.LsJob(grids_stub, lig, state(**over))])
    with pytest.raises(ValueError, match="shape"):
        dock.make_items([dock.LsJob(grids_stub, lig, state(), grad=torch.zeros(n, G - 1))])
    # Solis-Wets state, draws and scales
    def sw(**over):
        f = dict(genotype=torch.zeros(n, G), energy=torch.zeros(n), bias=torch.zeros(n, G),
                 rho=torch.ones(n), counts=torch.zeros(n, 2, dtype=torch.int32))
        f.update(over)
        return dock.SWState(**f)
    normals, scale = torch.zeros(3, n, G), torch.ones(G)
    with pytest.raises(ValueError, match="genes"):
        dock.solis_wets(grids_stub, lig, sw(genotype=torch.zeros(n, G - 1)), normals, scale)
    for over, what in ((dict(bias=torch.zeros(n, G + 1)), "shape"), (dict(rho=torch.ones(n + 1)), "shape"),
                       (dict(counts=torch.zeros(n, 2)), "int32"), ({}, "CUDA")):
        with pytest.raises(ValueError, match=what):
            dock.solis_wets(grids_stub, lig, sw(**over), normals, scale)
    with pytest.raises(ValueError, match="normals"):
        dock.solis_wets(grids_stub, lig, sw(), torch.zeros(3, n, G - 1), scale)
    with pytest.raises(ValueError):
        dock.score_batch(grids_stub, lig, torch.zeros(n, G - 1))
    with pytest.raises(ValueError, match="float32"):
        dock.score_batch(grids_stub, lig, torch.zeros(n, G, dtype=torch.float64))
