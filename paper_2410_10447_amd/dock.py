"""Python binding of the docking C ABI (include/dock.h), via ctypes.

Argument marshalling only: every computation runs in libdockmi.so. PyTorch is
used for device memory (tensors) and streams. The library must be built
(``python -m paper_2410_10447_amd.build_lib``); importing this module on a
machine without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

# DOCKMI_LIB names another build of the same ABI (the sanitizer build of
# the host code, libdockmi_san.so, for the CPU tests under ASan/UBSan)
_LIB_PATH = os.environ.get("DOCKMI_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                         "libdockmi.so")

# the struct layouts below follow include/dock.h of this ABI version
ABI_VERSION = 11

DOCK_OK = 0
DOCK_EINVAL = -1
DOCK_ENOMEM = -2
DOCK_EDEVICE = -3
DOCK_EUNSUPPORTED = -4

REDUCE_SHUFFLE = 0
REDUCE_MFMA_F32 = 1
REDUCE_MFMA_BF16 = 2
REDUCE_MFMA_F16 = 3
REDUCE_MFMA_BF16X3 = 4
REDUCE_SHARED_ATOMIC = 5
VARIANT_NAMES = {0: "shuffle", 1: "mfma_f32", 2: "mfma_bf16", 3: "mfma_f16", 4: "mfma_bf16x3",
                 5: "shared_atomic"}

LS_FINAL_EVAL = 1
LS_SEPARATE_LAUNCHES = 2
ITEM_PLAIN_MAPS = 1     # dock_ls_item.flags: read the planar maps
ITEM_TWO_PER_WAVE = 2   # dock_ls_item.flags: two individuals per wave (<= 32 atoms, <= 32 genes)
EXEC_TWO_PER_WAVE = 1   # dock_exec_opts.flags: two genotypes per wave
STATIC_MAX_ITEMS = 64   # items per dock_local_search_batch_static call

MAX_ATOMS = 128
MAX_TORSIONS = 32

# exported symbols of include/dock.h
ABI_SYMBOLS = (
    "dock_abi_version", "dock_last_error", "dock_create_grids", "dock_destroy_grids",
    "dock_grids_corner_bytes", "dock_grids_bind_corners",
    "dock_create_ligand", "dock_ligand_info_get", "dock_ligand_export", "dock_ligand_upload",
    "dock_destroy_ligand", "dock_score_batch", "dock_ls_workspace_bytes",
    "dock_select_rows", "dock_gather_rows", "dock_scatter_rows",
    "dock_local_search_batch", "dock_local_search_batch_static", "dock_ls_launches", "dock_block_sum4",
    "dock_ga_step", "dock_solis_wets_batch",
)


class DockError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"dock error {status}: {msg}")
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("n_maps", C.c_int32),
                ("spacing", C.c_float), ("origin", C.c_float * 3)]


class FFParams(C.Structure):
    _fields_ = [("n_classes", C.c_int32),
                ("radius", C.POINTER(C.c_double)), ("eps", C.POINTER(C.c_double)),
                ("solv", C.POINTER(C.c_double)), ("vol", C.POINTER(C.c_double)),
                ("donor", C.c_int32 * 2), ("acceptor", C.c_int32 * 2),
                ("hb_r0", (C.c_double * 2) * 2), ("hb_eps", (C.c_double * 2) * 2)]


class LigandDesc(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("n_torsions", C.c_int32), ("root_atom", C.c_int32),
                ("n_bonds", C.c_int32), ("xyz", C.POINTER(C.c_double)), ("charge", C.POINTER(C.c_double)),
                ("cls", C.POINTER(C.c_int32)), ("bonds", C.POINTER(C.c_int32)),
                ("rot_bonds", C.POINTER(C.c_int32)), ("ff", C.POINTER(FFParams))]


class LigandInfo(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("n_torsions", C.c_int32), ("n_genes", C.c_int32),
                ("n_pairs", C.c_int32), ("n_fragments", C.c_int32), ("max_depth", C.c_int32),
                ("n_batches", C.c_int32), ("n_copies", C.c_int32), ("blob_bytes", C.c_int64)]


class ExecOpts(C.Structure):
    _fields_ = [("variant", C.c_int32), ("threads_per_ind", C.c_int32), ("flags", C.c_uint32),
                ("atom_out", C.c_void_p)]


class LsItem(C.Structure):
    _fields_ = [("grids", C.c_void_p), ("ligand", C.c_void_p), ("n", C.c_int32),
                ("n_genes", C.c_int32), ("variant", C.c_int32), ("iterations", C.c_int32), ("final_eval", C.c_int32),
                ("threads_per_ind", C.c_int32),
                ("genotype", C.c_void_p), ("acc_g2", C.c_void_p), ("acc_dx2", C.c_void_p),
                ("best_genotype", C.c_void_p), ("best_energy", C.c_void_p),
                ("energy", C.c_void_p), ("iters_done", C.c_void_p), ("grad", C.c_void_p),
                ("flags", C.c_uint32)]


class LsOpts(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("rho", C.c_float), ("eps", C.c_float),
                ("variant", C.c_int32), ("threads_per_ind", C.c_int32), ("flags", C.c_uint32)]


class SwOpts(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("n_genes", C.c_int32), ("n_success", C.c_int32),
                ("n_failure", C.c_int32), ("variant", C.c_int32)]


class GaStepDesc(C.Structure):
    _fields_ = [("genotypes", C.c_void_p), ("energies", C.c_void_p), ("candidates", C.c_void_p),
                ("coins", C.c_void_p), ("cuts", C.c_void_p), ("mut_coin", C.c_void_p),
                ("mut_delta", C.c_void_p), ("children", C.c_void_p), ("best", C.c_void_p),
                ("n_runs", C.c_int32), ("pop", C.c_int32), ("n_genes", C.c_int32),
                ("p_tournament", C.c_float), ("p_crossover", C.c_float), ("p_mutation", C.c_float),
                ("elitism", C.c_int32)]


_lib = None


def lib():
    """Load libdockmi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with "
                          "`python -m paper_2410_10447_amd.build_lib`")
    L = C.CDLL(_LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    sig = {
        "dock_abi_version": ([], i32),
        "dock_last_error": ([], C.c_char_p),
        "dock_create_grids": ([C.POINTER(GridDesc), vp, C.POINTER(vp)], i32),
        "dock_destroy_grids": ([vp], i32),
        "dock_grids_corner_bytes": ([vp, C.POINTER(C.c_int64)], i32),
        "dock_grids_bind_corners": ([vp, vp, C.c_int64, vp], i32),
        "dock_create_ligand": ([C.POINTER(LigandDesc), C.POINTER(vp)], i32),
        "dock_ligand_info_get": ([vp, C.POINTER(LigandInfo)], i32),
        "dock_ligand_export": ([vp, vp, vp, vp, vp, vp, vp], i32),
        "dock_ligand_upload": ([vp, vp, vp], i32),
        "dock_destroy_ligand": ([vp], i32),
        "dock_score_batch": ([vp, vp, i32, vp, vp, vp, C.POINTER(ExecOpts), vp], i32),
        "dock_ls_workspace_bytes": ([i32, C.POINTER(i64)], i32),
        "dock_local_search_batch": ([C.POINTER(LsItem), i32, C.POINTER(LsOpts), vp, i64, vp], i32),
        "dock_local_search_batch_static": ([C.POINTER(LsItem), i32, C.POINTER(LsOpts), vp], i32),
        "dock_ls_launches": ([C.POINTER(LsItem), i32, C.POINTER(LsOpts), C.POINTER(i32)], i32),
        "dock_block_sum4": ([vp, vp, i32, i32, i32, i32, vp], i32),
        "dock_ga_step": ([C.POINTER(GaStepDesc), vp], i32),
        "dock_select_rows": ([vp, i32, C.c_float, vp, vp, vp], i32),
        "dock_gather_rows": ([vp, i32, i32, vp, i32, vp, vp], i32),
        "dock_scatter_rows": ([vp, i32, i32, vp, i32, vp, vp], i32),
        "dock_solis_wets_batch": ([vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, C.POINTER(SwOpts), vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    if L.dock_abi_version() != ABI_VERSION:
        raise ImportError(f"{_LIB_PATH} has ABI version {L.dock_abi_version()}, the binding "
                          f"expects {ABI_VERSION}: rebuild it")
    _lib = L
    return L


def _check(status):
    if status != DOCK_OK:
        raise DockError(status, lib().dock_last_error().decode())


def last_error() -> str:
    return lib().dock_last_error().decode()


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(None)


def _dptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _need(name, t, shape, dtype, device=None, placement=True):
    """Raise ValueError unless `t` is a contiguous CUDA tensor of the given
    shape and dtype (on `device` if given; the device checks only with
    `placement`): the C ABI receives bare pointers and cannot check any of
    this itself."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if not placement:
        return
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a CUDA tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name}: on {t.device}, expected {device}")


# ---------------------------------------------------------------------------
# Handles
# ---------------------------------------------------------------------------

class Grids:
    """Receptor grid set; `maps` is a float32 CUDA tensor [n_maps, nz, ny, nx]."""

    def __init__(self, maps, spacing: float, origin):
        import torch
        if not (isinstance(maps, torch.Tensor) and maps.is_cuda and maps.dtype == torch.float32
                and maps.dim() == 4 and maps.is_contiguous()):
            raise ValueError("maps must be a contiguous float32 CUDA tensor [M, nz, ny, nx]")
        self.maps = maps
        d = GridDesc()
        d.n_maps, d.nz, d.ny, d.nx = (int(v) for v in maps.shape)
        d.spacing = float(spacing)
        for c in range(3):
            d.origin[c] = float(origin[c])
        self.desc = d
        h = C.c_void_p()
        _check(lib().dock_create_grids(C.byref(d), _ptr(maps), C.byref(h)))
        self.handle = h
        self.corners = None

    @classmethod
    def from_synth(cls, g, device="cuda", corners: bool = True, stream=None):
        """Upload a synthetic grid set; with `corners` (the default) also build
        and bind the corner-expanded copy the kernels read fastest."""
        import torch
        G = cls(torch.from_numpy(np.ascontiguousarray(g.maps)).to(device), g.spacing, g.origin)
        if corners:
            G.bind_corners(stream=stream)
        return G

    def corner_bytes(self) -> int:
        n = C.c_int64()
        _check(lib().dock_grids_corner_bytes(self.handle, C.byref(n)))
        return int(n.value)

    def bind_corners(self, enable: bool = True, stream=None):
        """Build the corner-expanded copy (a uint8 CUDA tensor this object
        keeps) on `stream` and bind it; enable=False unbinds and frees it."""
        import torch
        if not enable:
            _check(lib().dock_grids_bind_corners(self.handle, None, 0, _stream_handle(stream)))
            self.corners = None
            return
        n = self.corner_bytes()
        buf = torch.empty(max(n, 16), dtype=torch.uint8, device=self.maps.device)
        _check(lib().dock_grids_bind_corners(self.handle, _ptr(buf), buf.numel(), _stream_handle(stream)))
        self.corners = buf

    def nbytes(self) -> int:
        return self.maps.numel() * 4 + (self.corners.numel() if self.corners is not None else 0)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.dock_destroy_grids(h)
            self.handle = None


def ff_params(ff):
    """Pack a synth.ForceField into the ABI struct (keeps the arrays alive)."""
    keep = [np.ascontiguousarray(a, dtype=np.float64) for a in (ff.radius, ff.eps, ff.solv, ff.vol)]
    p = FFParams()
    p.n_classes = len(keep[0])
    p.radius, p.eps, p.solv, p.vol = (_dptr(a, C.c_double) for a in keep)
    for i in range(2):
        p.donor[i] = int(ff.donors[i])
        p.acceptor[i] = int(ff.acceptors[i])
        for j in range(2):
            p.hb_r0[i][j] = float(ff.hb_r0[i, j])
            p.hb_eps[i][j] = float(ff.hb_eps[i, j])
    return p, keep


class Ligand:
    """Prepared ligand. `lig` has xyz, charge, cls, bonds ([n_bonds, 2]: a tree
    or a connected graph with rings), rot_bonds (indices into bonds), root."""

    def __init__(self, lig, ff, upload: bool = True, device="cuda"):
        xyz = np.ascontiguousarray(lig.xyz, dtype=np.float64)
        chg = np.ascontiguousarray(lig.charge, dtype=np.float64)
        cls = np.ascontiguousarray(lig.cls, dtype=np.int32)
        bonds = np.ascontiguousarray(np.asarray(lig.bonds, dtype=np.int32).reshape(-1, 2))
        rot = np.ascontiguousarray(lig.rot_bonds, dtype=np.int32)
        ffp, keep = ff_params(ff)
        d = LigandDesc()
        d.n_atoms = xyz.shape[0]
        d.n_torsions = rot.shape[0]
        d.root_atom = int(getattr(lig, "root", 0))
        d.n_bonds = bonds.shape[0]
        d.xyz = _dptr(xyz, C.c_double)
        d.charge = _dptr(chg, C.c_double)
        d.cls = _dptr(cls, C.c_int32)
        d.bonds = _dptr(bonds, C.c_int32)
        d.rot_bonds = _dptr(rot, C.c_int32)
        d.ff = C.pointer(ffp)
        h = C.c_void_p()
        _check(lib().dock_create_ligand(C.byref(d), C.byref(h)))
        del keep
        self.handle = h
        info = LigandInfo()
        _check(lib().dock_ligand_info_get(h, C.byref(info)))
        self.n_atoms = info.n_atoms
        self.n_torsions = info.n_torsions
        self.n_genes = info.n_genes
        self.n_pairs = info.n_pairs
        self.n_fragments = info.n_fragments
        self.max_depth = info.max_depth
        self.n_batches = info.n_batches
        self.n_copies = info.n_copies
        self.blob_bytes = info.blob_bytes
        self.blob = None
        if upload:
            self.upload(device)

    def upload(self, device="cuda", stream=None):
        import torch
        n = (self.blob_bytes + 15) // 16 * 16
        self.blob = torch.empty(n, dtype=torch.uint8, device=device)
        _check(lib().dock_ligand_upload(self.handle, _ptr(self.blob), _stream_handle(stream)))

    def export(self):
        N, T, P = self.n_atoms, self.n_torsions, self.n_pairs
        order = np.zeros(N, np.int32)
        tors = np.zeros((max(T, 1), 4), np.int32)
        frag = np.zeros(N, np.int32)
        pairs = np.zeros(max(P, 1), np.uint32)
        hb = np.zeros(max(P, 1), np.uint8)
        batches = np.zeros((max(self.n_batches, 1), 64), np.uint32)
        _check(lib().dock_ligand_export(self.handle, order.ctypes.data_as(C.c_void_p),
                                        tors.ctypes.data_as(C.c_void_p),
                                        frag.ctypes.data_as(C.c_void_p),
                                        pairs.ctypes.data_as(C.c_void_p),
                                        hb.ctypes.data_as(C.c_void_p),
                                        batches.ctypes.data_as(C.c_void_p)))
        pr = np.stack([pairs[:P] >> 16, pairs[:P] & 0xFFFF], axis=1).astype(np.int64)
        return {"order": order, "torsions": tors[:T], "fragment": frag, "pairs": pr,
                "pair_hb": hb[:P].astype(bool), "batches": batches[:self.n_batches]}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.dock_destroy_ligand(h)
            self.handle = None


# ---------------------------------------------------------------------------
# Batch calls
# ---------------------------------------------------------------------------

def score_batch(grids: Grids, ligand: Ligand, genotypes, variant: int = REDUCE_SHUFFLE,
                with_grad: bool = True, atom_out: bool = False, stream=None, two_per_wave: bool = False):
    """Energy [n] and gradient [n, G] of each genotype row (float32 CUDA tensor).
    `two_per_wave`: two genotypes per wave (ligands of <= 32 atoms and <= 32
    genes, the shuffle reduction)."""
    import torch
    if genotypes.dim() != 2 or genotypes.shape[1] != ligand.n_genes:
        raise ValueError(f"genotypes must be [n, {ligand.n_genes}]")
    n = genotypes.shape[0]
    gen = genotypes.contiguous()
    _need("genotypes", gen, (n, ligand.n_genes), torch.float32)
    E = torch.empty(n, dtype=torch.float32, device=gen.device)
    grad = torch.empty(n, ligand.n_genes, dtype=torch.float32, device=gen.device) if with_grad else None
    ao = torch.empty(n, ligand.n_atoms, 8, dtype=torch.float32, device=gen.device) if atom_out else None
    o = ExecOpts(variant=variant, threads_per_ind=0, flags=EXEC_TWO_PER_WAVE if two_per_wave else 0,
                 atom_out=(ao.data_ptr() if ao is not None else None))
    _check(lib().dock_score_batch(grids.handle, ligand.handle, n, _ptr(gen), _ptr(E), _ptr(grad),
                                  C.byref(o), _stream_handle(stream)))
    if atom_out:
        return E, grad, ao
    return E, grad


@dataclass
class LSState:
    """Device state of a local-search population (all CUDA tensors)."""
    genotype: object
    acc_g2: object
    acc_dx2: object
    best_genotype: object
    best_energy: object
    energy: object
    iters_done: object

    @classmethod
    def start(cls, genotypes):
        import torch
        g = genotypes.contiguous().clone()
        n = g.shape[0]
        return cls(g, torch.zeros_like(g), torch.zeros_like(g), g.clone(),
                   torch.full((n,), float("inf"), dtype=torch.float32, device=g.device),
                   torch.full((n,), float("nan"), dtype=torch.float32, device=g.device),
                   torch.zeros(n, dtype=torch.int32, device=g.device))

    def clone(self):
        return LSState(*(getattr(self, f).clone() for f in
                         ("genotype", "acc_g2", "acc_dx2", "best_genotype", "best_energy",
                          "energy", "iters_done")))

    def to_numpy(self):
        return {f: getattr(self, f).cpu().numpy() for f in
                ("genotype", "acc_g2", "acc_dx2", "best_genotype", "best_energy", "energy",
                 "iters_done")}

    def validate(self, n_genes: int):
        """Raise ValueError unless every tensor fits a population of rows of
        `n_genes` genes: [n, G] float32 rows, [n] float32 energies, [n] int32
        counts, all contiguous and on the genotype's device."""
        import torch
        g = self.genotype
        if not (isinstance(g, torch.Tensor) and g.dim() == 2):
            raise ValueError("LSState.genotype must be a 2-D tensor")
        n, dev = g.shape[0], g.device
        spec = [(f, (n, n_genes), torch.float32) for f in ("genotype", "acc_g2", "acc_dx2", "best_genotype")]
        spec += [(f, (n,), torch.float32) for f in ("best_energy", "energy")]
        spec += [("iters_done", (n,), torch.int32)]
        for placement in (False, True):      # every shape first, then placement
            for f, shp, dt in spec:
                _need(f"LSState.{f}", getattr(self, f), shp, dt, dev, placement)


def workspace_bytes(n_items: int) -> int:
    b = C.c_int64()
    _check(lib().dock_ls_workspace_bytes(n_items, C.byref(b)))
    return b.value


@dataclass
class LsJob:
    """One local-search item: a population of one ligand against one grid set.

    variant / iterations / final_eval of -1 defer to the call's options."""
    grids: object
    ligand: object
    state: object
    variant: int = -1
    iterations: int = -1
    final_eval: int = -1
    grad: object = None          # optional [n, G] CUDA tensor: gradient at the last evaluated point
    threads_per_ind: int = 0     # 64, 128 or 256, 0 defers to the call
    plain_maps: bool = False     # read the planar maps even with the corner copy bound
    two_per_wave: bool = False   # two individuals per wave (ligands of <= 32 atoms and <= 32 genes)


def _as_job(job):
    if isinstance(job, LsJob):
        return job
    return LsJob(*job)


def make_items(jobs):
    """jobs: LsJob or (Grids, Ligand, LSState[, variant[, iterations[, final_eval]]])."""
    arr = (LsItem * max(1, len(jobs)))()
    for i, job in enumerate(jobs):
        j = _as_job(job)
        grids, ligand, st = j.grids, j.ligand, j.state
        if j.grad is not None:
            import torch
            for placement in (False, True):
                _need("grad", j.grad, (st.genotype.shape[0], ligand.n_genes), torch.float32,
                      st.genotype.device, placement)
                if not placement:
                    st.validate(ligand.n_genes)
        else:
            st.validate(ligand.n_genes)
        it = arr[i]
        it.grids = grids.handle.value
        it.ligand = ligand.handle.value
        it.n = st.genotype.shape[0]
        it.n_genes = ligand.n_genes
        it.variant = j.variant
        it.iterations = j.iterations
        it.final_eval = j.final_eval
        it.threads_per_ind = j.threads_per_ind
        it.genotype = st.genotype.data_ptr()
        it.acc_g2 = st.acc_g2.data_ptr()
        it.acc_dx2 = st.acc_dx2.data_ptr()
        it.best_genotype = st.best_genotype.data_ptr()
        it.best_energy = st.best_energy.data_ptr()
        it.energy = st.energy.data_ptr()
        it.iters_done = st.iters_done.data_ptr()
        it.grad = j.grad.data_ptr() if j.grad is not None else None
        it.flags = (ITEM_PLAIN_MAPS if j.plain_maps else 0) | (ITEM_TWO_PER_WAVE if j.two_per_wave else 0)
    return arr


def local_search(jobs, iterations: int, rho: float = 0.8, eps: float = 1e-2,
                 variant: int = REDUCE_SHUFFLE, final_eval: bool = True, workspace=None,
                 stream=None, items=None, threads_per_ind: int = 0, separate_launches: bool = False):
    """ADADELTA on every (Grids, Ligand, LSState[, variant]) job, one call.

    State tensors are updated in place. `workspace` (uint8 CUDA tensor) is
    allocated if not given; `items` may pass a prebuilt item array.
    `threads_per_ind` (0/64/128/256) is the default for jobs that leave it at 0.
    `separate_launches` runs each kernel family in a launch of its own.
    """
    import torch
    n_items = len(jobs)
    if items is None:
        items = make_items(jobs)
    elif len(items) < n_items:
        raise ValueError("items shorter than jobs")
    need = workspace_bytes(n_items)
    if workspace is None or workspace.numel() < need:
        dev = torch.device("cuda")
        workspace = torch.empty(max(need, 64), dtype=torch.uint8, device=dev)
    o = LsOpts(iterations=iterations, rho=rho, eps=eps, variant=variant, threads_per_ind=threads_per_ind,
               flags=(LS_FINAL_EVAL if final_eval else 0) | (LS_SEPARATE_LAUNCHES if separate_launches else 0))
    _check(lib().dock_local_search_batch(items, n_items, C.byref(o), _ptr(workspace),
                                         workspace.numel(), _stream_handle(stream)))
    return workspace


def ls_launches(jobs, iterations: int, variant: int = REDUCE_SHUFFLE, final_eval: bool = True,
                threads_per_ind: int = 0, separate_launches: bool = False, items=None) -> int:
    """Persistent launches local_search would make for these jobs."""
    n_items = len(jobs)
    if items is None:
        items = make_items(jobs)
    elif len(items) < n_items:
        raise ValueError("items shorter than jobs")
    o = LsOpts(iterations=iterations, rho=0.8, eps=1e-2, variant=variant, threads_per_ind=threads_per_ind,
               flags=(LS_FINAL_EVAL if final_eval else 0) | (LS_SEPARATE_LAUNCHES if separate_launches else 0))
    n = C.c_int32(0)
    _check(lib().dock_ls_launches(items, n_items, C.byref(o), C.byref(n)))
    return n.value


def local_search_static(jobs, iterations: int, rho: float = 0.8, eps: float = 1e-2,
                        variant: int = REDUCE_SHUFFLE, final_eval: bool = True, stream=None,
                        items=None, threads_per_ind: int = 0, separate_launches: bool = False):
    """local_search through dock_local_search_batch_static: the workspace is
    the library's own (at most STATIC_MAX_ITEMS jobs per call); the call
    allocates no device memory. Calls that may overlap on one GPU race."""
    n_items = len(jobs)
    if items is None:
        items = make_items(jobs)
    elif len(items) < n_items:
        raise ValueError("items shorter than jobs")
    o = LsOpts(iterations=iterations, rho=rho, eps=eps, variant=variant, threads_per_ind=threads_per_ind,
               flags=(LS_FINAL_EVAL if final_eval else 0) | (LS_SEPARATE_LAUNCHES if separate_launches else 0))
    _check(lib().dock_local_search_batch_static(items, n_items, C.byref(o), _stream_handle(stream)))


def block_sum4(x, variant: int, repeat: int = 1, stream=None):
    """x: float32 CUDA tensor [n_blocks, threads, 4] -> every thread's block total."""
    import torch
    nb, th, four = x.shape
    assert four == 4
    x = x.contiguous()
    out = torch.empty_like(x)
    _check(lib().dock_block_sum4(_ptr(x), _ptr(out), nb, th, variant, repeat, _stream_handle(stream)))
    return out


def ga_step(genotypes, energies, candidates, coins, cuts, mut_coin, mut_delta,
            p_tournament: float, p_crossover: float, p_mutation: float, elitism: bool,
            children=None, best=None, stream=None):
    """One GA generation step (dock_ga_step) on CUDA tensors.

    genotypes (R, P, G) float32, energies (R, P) float32, candidates (R, P, 4)
    int32, coins (R, P, 3) float32, cuts (R, P, 2) int32, mut_coin and
    mut_delta (R, P, G) float32. Returns (children (R, P, G), best (R,) int32).
    """
    import torch
    R, P, G = genotypes.shape
    args = [t.contiguous() for t in (genotypes, energies, candidates, coins, cuts, mut_coin, mut_delta)]
    gen, E, cand, cn, cu, mc, md = args
    shapes = {"energies": (E, (R, P), torch.float32), "candidates": (cand, (R, P, 4), torch.int32),
              "coins": (cn, (R, P, 3), torch.float32), "cuts": (cu, (R, P, 2), torch.int32),
              "mut_coin": (mc, (R, P, G), torch.float32), "mut_delta": (md, (R, P, G), torch.float32)}
    if gen.dtype != torch.float32:
        raise ValueError("genotypes must be float32")
    for name, (t, shp, dt) in shapes.items():
        if tuple(t.shape) != shp or t.dtype != dt:
            raise ValueError(f"{name}: expected {shp} {dt}, got {tuple(t.shape)} {t.dtype}")
    if children is None:
        children = torch.empty_like(gen)
    if best is None:
        best = torch.empty(R, dtype=torch.int32, device=gen.device)
    d = GaStepDesc(_ptr(gen).value, _ptr(E).value, _ptr(cand).value, _ptr(cn).value, _ptr(cu).value,
                   _ptr(mc).value, _ptr(md).value, _ptr(children).value, _ptr(best).value,
                   R, P, G, float(p_tournament), float(p_crossover), float(p_mutation), int(bool(elitism)))
    _check(lib().dock_ga_step(C.byref(d), _stream_handle(stream)))
    return children, best


def select_rows(draws, rate: float, index=None, count=None, stream=None):
    """Rows with draws[r] < rate, increasing (dock_select_rows): returns
    (index [n] int32, count [1] int32), CUDA tensors; index[:count] holds
    the rows."""
    import torch
    n = draws.shape[0]
    d = draws.contiguous()
    _need("draws", d, (n,), torch.float32)
    if index is None:
        index = torch.empty(max(n, 1), dtype=torch.int32, device=d.device)
    if count is None:
        count = torch.empty(1, dtype=torch.int32, device=d.device)
    _need("index", index, (max(n, 1),), torch.int32, d.device)
    _need("count", count, (1,), torch.int32, d.device)
    _check(lib().dock_select_rows(_ptr(d), n, float(rate), _ptr(index), _ptr(count), _stream_handle(stream)))
    return index, count


def _rows(t):
    return t.shape[0], (int(np.prod(t.shape[1:])) if t.dim() > 1 else 1)


def gather_rows(src, index, m: int, stream=None):
    """dst[k] = src[index[k]] for k < m (dock_gather_rows); src [n, ...] float32."""
    import torch
    s = src.contiguous()
    if s.dtype != torch.float32:
        raise ValueError("src must be float32")
    n, row = _rows(s)
    if index.dtype != torch.int32 or not index.is_contiguous() or index.shape[0] < m:
        raise ValueError("index must be a contiguous int32 tensor of at least m entries")
    dst = torch.empty((m,) + tuple(s.shape[1:]), dtype=torch.float32, device=s.device)
    _check(lib().dock_gather_rows(_ptr(s), n, row, _ptr(index), m, _ptr(dst), _stream_handle(stream)))
    return dst


def scatter_rows(src, index, dst, stream=None):
    """dst[index[k]] = src[k] for k < len(src), in place (dock_scatter_rows)."""
    import torch
    s = src.contiguous()
    m, row = _rows(s)
    n, row_d = _rows(dst)
    if s.dtype != torch.float32 or dst.dtype != torch.float32 or row != row_d or not dst.is_contiguous():
        raise ValueError("src and dst must be float32 with rows of the same size (dst contiguous)")
    if index.dtype != torch.int32 or not index.is_contiguous() or index.shape[0] < m:
        raise ValueError("index must be a contiguous int32 tensor of at least len(src) entries")
    _check(lib().dock_scatter_rows(_ptr(s), m, row, _ptr(index), n, _ptr(dst), _stream_handle(stream)))
    return dst


def ga_draws(n_runs: int, pop: int, n_genes: int, generator, device,
             max_translation: float = 2.0, max_quaternion: float = 0.25, max_torsion: float = 1.5708):
    """Random inputs of one GA step, drawn on the device with a seeded torch
    generator: tournament candidates, coins, cut points, mutation draws, and
    displacements uniform in +-max_translation (genes 0..2, Angstrom),
    +-max_quaternion (genes 3..6) and +-max_torsion (torsion genes, rad)."""
    import torch
    R, P, G = n_runs, pop, n_genes
    kw = dict(generator=generator, device=device)
    cand = torch.randint(0, P, (R, P, 4), dtype=torch.int32, **kw)
    coins = torch.rand((R, P, 3), dtype=torch.float32, **kw)
    cuts = torch.randint(0, G + 1, (R, P, 2), dtype=torch.int32, **kw)
    mut_coin = torch.rand((R, P, G), dtype=torch.float32, **kw)
    scale = torch.full((G,), max_torsion, dtype=torch.float32, device=device)
    scale[:3] = max_translation
    scale[3:7] = max_quaternion
    mut_delta = (torch.rand((R, P, G), dtype=torch.float32, **kw) * 2.0 - 1.0) * scale
    return cand, coins, cuts, mut_coin, mut_delta


@dataclass
class SWState:
    """Device state of a Solis-Wets population (CUDA tensors)."""
    genotype: object     # [n, G] float32
    energy: object       # [n] float32, energy of genotype
    bias: object         # [n, G] float32
    rho: object          # [n] float32
    counts: object       # [n, 2] int32: successes, failures in a row

    @classmethod
    def start(cls, genotypes, energies, rho0: float = 1.0):
        import torch
        g = genotypes.contiguous().clone()
        n = g.shape[0]
        return cls(g, energies.contiguous().clone(), torch.zeros_like(g),
                   torch.full((n,), rho0, dtype=torch.float32, device=g.device),
                   torch.zeros((n, 2), dtype=torch.int32, device=g.device))


def solis_wets(grids: Grids, ligand: Ligand, st: SWState, normals, scale, n_success: int = 4,
               n_failure: int = 4, variant: int = REDUCE_SHUFFLE, log: bool = False, stream=None):
    """len(normals) Solis-Wets iterations in place on `st` (dock_solis_wets_batch).
    normals [iters, n, G] float32, scale [G] float32 (CUDA tensors). Returns the
    trials' energies [n, iters, 2] if `log`, else None."""
    import torch
    iters = normals.shape[0]
    if st.genotype.dim() != 2:
        raise ValueError("SWState.genotype must be [n, G]")
    n, G = st.genotype.shape
    if G != ligand.n_genes:
        raise ValueError(f"SWState rows have {G} genes, the ligand {ligand.n_genes}")
    dev = st.genotype.device
    spec = (("genotype", (n, G), torch.float32), ("energy", (n,), torch.float32),
            ("bias", (n, G), torch.float32), ("rho", (n,), torch.float32),
            ("counts", (n, 2), torch.int32))
    if tuple(normals.shape[1:]) != (n, G) or tuple(scale.shape) != (G,):
        raise ValueError("normals must be [iters, n, G] and scale [G]")
    nm = normals.contiguous()
    sc = scale.contiguous()
    for placement in (False, True):          # every shape first, then placement
        for f, shp, dt in spec:
            _need(f"SWState.{f}", getattr(st, f), shp, dt, dev, placement)
        _need("normals", nm, (iters, n, G), torch.float32, dev, placement)
        _need("scale", sc, (G,), torch.float32, dev, placement)
    lg = torch.empty((n, iters, 2), dtype=torch.float32, device=dev) if log else None
    o = SwOpts(iters, G, n_success, n_failure, variant)
    _check(lib().dock_solis_wets_batch(grids.handle, ligand.handle, n, _ptr(st.genotype), _ptr(st.energy),
                                       _ptr(st.bias), _ptr(st.rho), _ptr(st.counts), _ptr(nm), _ptr(sc),
                                       C.byref(o), _ptr(lg), _stream_handle(stream)))
    return lg
