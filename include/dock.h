/*
 * dock.h - C ABI of the MI355X docking hot path.
 *
 * The library evaluates the scoring function of a flexible ligand against a
 * fixed receptor (energy and analytic gradient with respect to the genotype)
 * for batches of individuals, and runs the ADADELTA local search of a
 * Lamarckian genetic algorithm on them (Sec. 2.1 of "Accelerating Drug
 * Discovery in AutoDock-GPU with Tensor Cores": the receptor is fixed, a pose
 * is the genotype {position, orientation, torsion angles}, each local-search
 * iteration needs E and its gradient, built from block-level sums of the
 * energy, the Cartesian gradient and the torque). The block sum of
 * {E, gx, gy, gz} (Sec. 3 and Sec. 4.2) is selectable between a wavefront
 * shuffle reduction and matrix-core (MFMA) contractions.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an int32 status (DOCK_OK or a negative DOCK_E*)
 *   and never aborts or throws. dock_last_error() returns a thread-local,
 *   human-readable description of the last failure on the calling thread.
 * - Argument and shape validation is synchronous and happens before any
 *   device work is enqueued; a failing call enqueues nothing.
 * - Batch calls are asynchronous on the HIP stream passed as `stream`
 *   (a hipStream_t; NULL is the null stream). Launch failures are reported
 *   immediately as DOCK_EDEVICE; faults during execution surface on the next
 *   synchronising call (through HIP or the caller's framework).
 * - "host" pointers are read during the call only and may be freed when it
 *   returns. "device" pointers are borrowed: the caller owns them and keeps
 *   them alive until the stream work that uses them has completed.
 * - Genotype layout (float32, row-major, G = 7 + T genes per individual):
 *   [tx, ty, tz, qw, qx, qy, qz, psi_1 .. psi_T]: translation (A), a
 *   quaternion (normalised on use), torsion angles (rad). Gradients use the
 *   same layout.
 * - Non-finite genotypes propagate to non-finite outputs; there is no
 *   device-side error channel.
 */
#ifndef DOCK_H
#define DOCK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DOCK_ABI_VERSION 11

/* status codes */
#define DOCK_OK            0
#define DOCK_EINVAL       (-1)  /* bad argument, shape or size */
#define DOCK_ENOMEM       (-2)  /* host allocation failed */
#define DOCK_EDEVICE      (-3)  /* HIP runtime error or launch failure */
#define DOCK_EUNSUPPORTED (-4)  /* valid request outside the built limits */

/* limits of this build */
#define DOCK_MAX_ATOMS     128
#define DOCK_MAX_TORSIONS   32
#define DOCK_MAX_GENES     (7 + DOCK_MAX_TORSIONS)
#define DOCK_MAX_CLASSES    32

/* block-sum variants for {E, gx, gy, gz} (Sec. 3 baseline, Sec. 4.2 method) */
#define DOCK_REDUCE_SHUFFLE   0  /* wave64 cross-lane (DPP) butterfly, FP32 */
#define DOCK_REDUCE_MFMA_F32  1  /* FP32 MFMA 16x16x4 with a 0/1 selection matrix */
#define DOCK_REDUCE_MFMA_BF16 2  /* BF16 MFMA 16x16x32, hi/lo split, FP32 accumulate */
#define DOCK_REDUCE_MFMA_F16  3  /* FP16 MFMA 16x16x32, scaled hi/lo split, FP32 accumulate */
#define DOCK_REDUCE_MFMA_BF16X3 4 /* BF16 MFMA, hi/mid/lo split (3 terms), FP32 accumulate */
#define DOCK_REDUCE_COUNT     5  /* variants usable by the scoring and search calls */
#define DOCK_REDUCE_SHARED_ATOMIC 5 /* dock_block_sum4 only: the Sec. 3 baseline, per
                                       component a shuffle tree, one LDS atomic per wave
                                       and three barriers */

int32_t dock_abi_version(void);

/* Text of the last error on the calling thread ("" if none). The pointer
 * stays valid until the next failing call on the same thread. */
const char* dock_last_error(void);

/* ------------------------------------------------------------------------
 * Receptor grids (Sec. 2.1: the target molecule is fixed, so its
 * interaction with each ligand atom type is precomputed on a lattice).
 * ---------------------------------------------------------------------- */
typedef struct dock_grids dock_grids;

typedef struct {
    int32_t nx, ny, nz;  /* nodes per axis, each >= 2 */
    int32_t n_maps;      /* >= 3: atom-type maps [0, n_maps-2), then the
                            electrostatic map (scaled by the atom charge), then
                            the desolvation map (scaled by |charge|) */
    float spacing;       /* lattice spacing h (A), > 0 */
    float origin[3];     /* position of node (0,0,0) (A), (x, y, z) */
} dock_grid_desc;

/* maps_dev: device, float32 [n_maps][nz][ny][nx] (x fastest), borrowed for the
 * lifetime of the handle, 4-byte aligned. Errors: DOCK_EINVAL on NULL
 * pointers, non-positive sizes or spacing, n_maps < 3. */
int32_t dock_create_grids(const dock_grid_desc* desc, const float* maps_dev, dock_grids** out);
/* NULL is accepted (DOCK_OK). */
int32_t dock_destroy_grids(dock_grids* grids);

/* Corner-expanded copy of the maps, for the trilinear term of Sec. 2.1
 * (each atom reads the 8 corners of its cell in its type map, the
 * electrostatic and the desolvation map): for every atom type t < n_maps-2
 * and every cell (cx, cy, cz) of the (nx-1)(ny-1)(nz-1) cells (x fastest),
 * the cell's 8 corner values v[4 dz + 2 dy + dx] of map t, of the
 * electrostatic and of the desolvation map, as 96 contiguous bytes of a
 * 128-byte block (32 bytes of zeros). An atom then reads one block (one
 * cache line when the buffer is 128-byte aligned) instead of twelve separate
 * rows; the values and the arithmetic are the same, so scores are identical
 * with and without it. *bytes = (n_maps-2) (nx-1)(ny-1)(nz-1) 128 (about
 * 32 (n_maps-2)/n_maps times the maps). */
int32_t dock_grids_corner_bytes(const dock_grids* grids, int64_t* bytes);
/* Fills corners_dev (device, caller-owned, 16-byte aligned, >= the size above)
 * from the handle's maps on `stream` and binds it to the handle: later calls
 * read it (so they must run on `stream` or after it); the maps stay borrowed.
 * corners_dev = NULL unbinds (the maps are read directly). Errors:
 * DOCK_EINVAL for a NULL handle, a small or misaligned buffer (no device work
 * is started then). */
int32_t dock_grids_bind_corners(dock_grids* grids, void* corners_dev, int64_t bytes, void* stream);

/* ------------------------------------------------------------------------
 * Ligand: topology, torsion tree and intramolecular pair list, prepared once
 * on the host (Sec. 2.1: N_rot torsion genes act on rotatable bonds; the
 * score sums pairwise interactions).
 * ---------------------------------------------------------------------- */
typedef struct dock_ligand dock_ligand;

typedef struct {
    int32_t n_classes;        /* entries in each per-class array, <= DOCK_MAX_CLASSES */
    const double* radius;     /* host [n_classes]: vdW radius R (A); r0 = R_i + R_j */
    const double* eps;        /* host [n_classes]: well depth; eps_ij = sqrt(eps_i eps_j) */
    const double* solv;       /* host [n_classes]: solvation parameter s */
    const double* vol;        /* host [n_classes]: atomic volume V (A^3) */
    int32_t donor[2];         /* classes that donate a hydrogen bond */
    int32_t acceptor[2];      /* classes that accept one */
    double hb_r0[2][2];       /* [donor][acceptor] 12-10 equilibrium distance (A) */
    double hb_eps[2][2];      /* [donor][acceptor] 12-10 well depth */
} dock_ff_params;

typedef struct {
    int32_t n_atoms;          /* 1 .. DOCK_MAX_ATOMS */
    int32_t n_torsions;       /* 0 .. DOCK_MAX_TORSIONS */
    int32_t root_atom;        /* atom that stays on the fixed side of every torsion */
    int32_t n_bonds;          /* n_atoms - 1 (a tree) .. 4 n_atoms (rings) */
    const double* xyz;        /* host [n_atoms][3] reference conformation (A) */
    const double* charge;     /* host [n_atoms] partial charges (e) */
    const int32_t* cls;       /* host [n_atoms] classes, < ff->n_classes */
    const int32_t* bonds;     /* host [n_bonds][2]: the bond graph, connected; rings
                                 stay inside rigid fragments */
    const int32_t* rot_bonds; /* host [n_torsions]: indices into bonds; each an
                                 internal bond (both ends bonded elsewhere) that
                                 lies in no ring */
    const dock_ff_params* ff; /* host */
} dock_ligand_desc;

typedef struct {
    int32_t n_atoms, n_torsions, n_genes;
    int32_t n_pairs;          /* intramolecular pairs kept */
    int32_t n_fragments;      /* rigid fragments = n_torsions + 1 */
    int32_t max_depth;        /* longest chain of nested torsions */
    int32_t n_batches;        /* 64-wide batches the pair list is cut into */
    int32_t n_copies;         /* force accumulator copies per atom (see export) */
    int64_t blob_bytes;       /* device bytes needed by dock_ligand_upload */
} dock_ligand_info;

/* Prepares the ligand on the host (no device call). The preparation orders
 * atoms depth-first from the root (neighbours by increasing index), turns
 * each rotatable bond into a torsion whose moving atoms (the side of the bond
 * away from the root) form one contiguous range of that order, splits the
 * molecule into rigid fragments (rings stay inside one), and keeps the atom
 * pairs that are >= 4 bonds apart (shortest path in the bond graph) and in
 * different fragments. Errors: DOCK_EINVAL if the bonds do not connect the
 * n_atoms atoms, repeat a bond, or n_bonds is outside [n_atoms - 1,
 * 4 n_atoms]; a rotatable bond is not internal, lies in a ring or is
 * repeated; a class is out of range; DOCK_EUNSUPPORTED beyond the build
 * limits. */
int32_t dock_create_ligand(const dock_ligand_desc* desc, dock_ligand** out);
int32_t dock_ligand_info_get(const dock_ligand* lig, dock_ligand_info* out);

/* Host copies of the prepared topology, decoded from the packed data the
 * kernels read. Any output may be NULL.
 *   order     [n_atoms]        atom index at each depth-first position
 *   torsions  [n_torsions][4]  (a, b, first, end): bond a->b (a on the root
 *                              side, original indices) and the half-open range
 *                              of depth-first positions that the torsion moves
 *   fragment  [n_atoms]        fragment id of each atom (0 = root fragment,
 *                              k+1 = the fragment next to torsion k's b atom)
 *   pairs     [n_pairs]        (i << 16) | j with i < j (original indices),
 *                              sorted ascending
 *   pair_hb   [n_pairs]        1 for a donor-acceptor (12-10) pair, else 0
 *   batches   [n_batches][64]  the pair list as the kernels read it, decoded: one
 *                              record per lane, i | j << 7 | ci << 14 | cj << 18 |
 *                              hb << 22 | valid << 31, with i, j depth-first
 *                              positions and ci, cj < n_copies the accumulator
 *                              copies the pair's force goes to; within a batch
 *                              every (copy, atom) slot occurs at most once. An
 *                              unused lane (valid clear) holds two slots no pair
 *                              of its batch uses; its i, j may be "atoms" past
 *                              n_atoms (below the next power of two, at least 16)
 *                              whose slots are never summed */
int32_t dock_ligand_export(const dock_ligand* lig, int32_t* order, int32_t* torsions,
                           int32_t* fragment, uint32_t* pairs, uint8_t* pair_hb,
                           uint32_t* batches);

/* Copies the packed ligand (blob_bytes, see dock_ligand_info) to blob_dev
 * (device, caller-owned, 16-byte aligned) asynchronously on `stream` (staged
 * through library-owned pinned memory, so the call does not wait for the
 * device) and binds it to the handle: later batch calls read the ligand from
 * there, so they must run on the same stream or after it. Call again to
 * rebind. */
int32_t dock_ligand_upload(dock_ligand* lig, void* blob_dev, void* stream);
int32_t dock_destroy_ligand(dock_ligand* lig);

/* ------------------------------------------------------------------------
 * One scoring evaluation per individual: energy and gradient (Sec. 2.1).
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t variant;          /* DOCK_REDUCE_* */
    int32_t threads_per_ind;  /* 0 (= 64) or 64; wider tiles are reserved */
    uint32_t flags;           /* 0, or DOCK_EXEC_TWO_PER_WAVE */
    float* atom_out;          /* device [n][n_atoms][8] or NULL: per atom (original
                                 order) x - tx, y - ty, z - tz (the atom's position
                                 relative to the translation genes, the FP32 values
                                 the evaluation holds: t plus these, summed exactly,
                                 is the world position its terms use), e_inter (the
                                 atom's grid energy with the outside penalty),
                                 gx, gy, gz (dE/dx of the atom), 0 */
} dock_exec_opts;

/* Scoring flag: two genotypes per wave (see DOCK_ITEM_TWO_PER_WAVE; same
 * requirements: <= 32 atoms and <= 32 genes, the shuffle reduction). */
#define DOCK_EXEC_TWO_PER_WAVE 1u

/* genotypes_dev [n][G], energy_dev [n], grad_dev [n][G] (may be NULL): device
 * float32, 4-byte aligned. opts may be NULL (defaults). Errors: DOCK_EINVAL on
 * NULL handles or pointers, n < 0, a ligand that was never uploaded, a
 * ligand class with no type map; n == 0 is a no-op. */
int32_t dock_score_batch(const dock_grids* grids, const dock_ligand* lig, int32_t n,
                         const float* genotypes_dev, float* energy_dev, float* grad_dev,
                         const dock_exec_opts* opts, void* stream);

/* ------------------------------------------------------------------------
 * ADADELTA local search (Sec. 2.1; Zeiler 2012), many ligands in one launch.
 * Each iteration evaluates E and dE/dgenotype at the current point, records
 * the point if E is the lowest seen so far (first minimum wins ties), and
 * takes one ADADELTA step on every gene; the quaternion is renormalised after
 * each step (kept if its norm falls below 1e-6).
 * ---------------------------------------------------------------------- */
typedef struct {
    const dock_grids* grids;
    const dock_ligand* ligand;   /* uploaded */
    int32_t n;                   /* individuals in this item, >= 0 */
    int32_t n_genes;             /* G of the rows below; must equal the ligand's 7 + T */
    int32_t variant;             /* DOCK_REDUCE_* for this item, or -1 = opts->variant */
    int32_t iterations;          /* steps for this item, 0 .. opts->iterations, or -1 = opts */
    int32_t final_eval;          /* 1/0 overrides DOCK_LS_FINAL_EVAL for this item, -1 = opts */
    int32_t threads_per_ind;     /* 64, 128 or 256 for this item, 0 = opts->threads_per_ind */
    float* genotype;             /* device [n][G] in/out: current point */
    float* acc_g2;               /* device [n][G] in/out: running mean of g^2 (start 0) */
    float* acc_dx2;              /* device [n][G] in/out: running mean of dx^2 (start 0) */
    float* best_genotype;        /* device [n][G] in/out */
    float* best_energy;          /* device [n] in/out (start +inf) */
    float* energy;               /* device [n] out: E at the last evaluated point */
    int32_t* iters_done;         /* device [n] in/out: iterations taken so far */
    float* grad;                 /* device [n][G] out, or NULL: dE/dgenotype at the last
                                    evaluated point */
    uint32_t flags;              /* DOCK_ITEM_PLAIN_MAPS | DOCK_ITEM_TWO_PER_WAVE, or 0 */
} dock_ls_item;

/* Item flag: read the planar maps even when the grid set has the
 * corner-expanded copy bound (a layout choice per item, e.g. per size
 * bucket of a tuning table; the values, and so the results, are the same). */
#define DOCK_ITEM_PLAIN_MAPS 1u
/* Item flag: two individuals per wave, one per 32-lane half (individuals
 * 2k and 2k + 1 of the item share a wave; their results do not depend on
 * each other). Needs a ligand of at most 32 atoms and 32 genes, the
 * shuffle reduction and one wave per individual (threads_per_ind 0 or 64),
 * else DOCK_EUNSUPPORTED. The block sum runs over each half, so results
 * differ from one individual per wave by rounding only. */
#define DOCK_ITEM_TWO_PER_WAVE 2u

#define DOCK_LS_FINAL_EVAL 1u    /* evaluate the point reached after the last step */
/* Run every kernel family in a launch of its own, even where they could
 * share one (see dock_local_search_batch); the results are the same. */
#define DOCK_LS_SEPARATE_LAUNCHES 2u

typedef struct {
    int32_t iterations;          /* >= 0 steps per individual in this call */
    float rho;                   /* decay, 0 < rho < 1 (0.8) */
    float eps;                   /* conditioner, > 0 (1e-2) */
    int32_t variant;             /* default DOCK_REDUCE_* */
    int32_t threads_per_ind;     /* 0 (= 64), 64, 128 or 256: threads (waves of 64)
                                    per individual; with 128 or 256 the waves split
                                    the pair batches (and, past 64 atoms, the first
                                    two waves the atoms) */
    uint32_t flags;              /* DOCK_LS_FINAL_EVAL | DOCK_LS_SEPARATE_LAUNCHES */
} dock_ls_opts;

/* Device bytes of the workspace dock_local_search_batch needs for n_items. */
int32_t dock_ls_workspace_bytes(int32_t n_items, int64_t* bytes);

/* Runs opts->iterations steps (or the item's own count) on every individual
 * of every item in one persistent launch; items are scheduled longest first.
 * Items run in up to five kernel families: ligands of <= 64 atoms (one
 * wave per individual), larger ligands with one wave (two atoms per lane),
 * any ligand with two or four waves per individual (128 or 256 threads: wave
 * w owns atoms 64 w .. 64 w + 63, if the ligand has them, and the w-th run
 * of ceil(batches / waves) pair batches), or two individuals per wave
 * (DOCK_ITEM_TWO_PER_WAVE). A batch that mixes families still runs as one
 * persistent launch when every item uses one reduction variant and either
 * (a) its families are among two waves per individual, one wave for a
 * ligand of <= 64 atoms, and two per wave, and every item reads the
 * corner-expanded maps (128-thread blocks: most blocks take two-wave
 * individuals first, the rest, sized by the estimated share of the work,
 * start on one-wave units, which each wave of a block takes on its own), or
 * (b) they are the two one-wave families (the kernel picks the atom layout
 * per item).
 * Otherwise, or with DOCK_LS_SEPARATE_LAUNCHES, it runs as one persistent
 * launch per family, side by side: the first on `stream`, the others on
 * streams the library owns (per device), forked from and joined back into
 * `stream` with events, so work queued on `stream` after the call still
 * waits for all of them. Every item's results are the same bit for bit
 * whichever way it runs.
 * Items may be at different stages: a serving loop passes each job's
 * remaining steps and asks for the final evaluation only in its last call. A call of K
 * iterations without DOCK_LS_FINAL_EVAL followed by one with it gives the
 * same state, bit for bit, as a single call with all the iterations.
 * workspace_dev: device, >= dock_ls_workspace_bytes(n_items), 16-byte
 * aligned, caller-owned; it must not be shared by calls that may overlap.
 * Errors: DOCK_EINVAL on NULL pointers, bad opts, an item whose n_genes is not
 * its ligand's gene count, a ligand never uploaded, or a workspace that is
 * too small. */
int32_t dock_local_search_batch(const dock_ls_item* items, int32_t n_items,
                                const dock_ls_opts* opts, void* workspace_dev,
                                int64_t workspace_bytes, void* stream);

/* The number of persistent launches dock_local_search_batch would make for
 * these items and opts (0 when no item has work): the same validation, no
 * device work, no allocation on the device. */
int32_t dock_ls_launches(const dock_ls_item* items, int32_t n_items, const dock_ls_opts* opts,
                         int32_t* n_launches);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * search as dock_local_search_batch, same items, opts, kernels and results
 * bit for bit, with the workspace held by the library instead of passed in.
 * Each GPU holds one library-resident workspace of
 * 64 + DOCK_STATIC_MAX_ITEMS item records (about 11 KB) until the process
 * ends; the call writes its item table there with kernel launches on
 * `stream` (the data travels in kernel arguments) and then launches the
 * search on `stream`, each kernel family after the other (no side streams).
 * It calls no hipMalloc, hipFree, hipHostMalloc or memset/memcpy: only
 * kernel launches. Every call on one GPU shares that workspace, so calls
 * that may overlap on one GPU (different streams, or different host
 * threads) race and must not be made; calls queued on one stream are safe.
 * Errors: those of dock_local_search_batch, and DOCK_EINVAL for more than
 * DOCK_STATIC_MAX_ITEMS items (nothing is launched then). */
#define DOCK_STATIC_MAX_ITEMS 64
int32_t dock_local_search_batch_static(const dock_ls_item* items, int32_t n_items,
                                       const dock_ls_opts* opts, void* stream);

/* ------------------------------------------------------------------------
 * Isolated block sum (the paper's reduction test kernel, Sec. 5.2): each of
 * the `threads` threads of each block holds one float4; every thread ends
 * with the block total. in_dev [n_blocks][threads][4], out_dev
 * [n_blocks][threads][4] (every thread's copy of the total), device float32.
 * threads: 64 .. 1024, a multiple of 64. variant: DOCK_REDUCE_* or
 * DOCK_REDUCE_SHARED_ATOMIC. repeat >= 1 runs the reduction that many times
 * in a dependent chain inside the kernel (timing).
 * ---------------------------------------------------------------------- */
int32_t dock_block_sum4(const float* in_dev, float* out_dev, int32_t n_blocks, int32_t threads,
                        int32_t variant, int32_t repeat, void* stream);

/* ------------------------------------------------------------------------
 * Solis-Wets local search (Sec. 2.1: the LGA's second local search beside
 * ADADELTA; it needs energies only). The paper gives no step; this is the
 * random search of Solis and Wets as AutoDock uses it. Per iteration and
 * individual, with z the iteration's standard normal draws (an input):
 *   dev = rho * (scale[g] * z[g]);
 *   trial 1: x + bias + dev; if E < current: move, bias = 0.2 bias + 0.4 dev;
 *   else trial 2: x - bias - dev; if E < current: move, bias = bias - 0.4 dev;
 *   else bias = 0.5 bias (a failure);
 *   n_success successes in a row double rho, n_failure failures halve it.
 * Float32 throughout, every state update in the order written with no fused
 * operations; one wave per individual (ligands of up to DOCK_MAX_ATOMS
 * atoms), the energy by the scoring evaluation with the chosen FP32 variant.
 * Device arrays, float32 unless stated, row-major, caller-owned, in/out:
 *   genotype [n][G], energy [n] (the energy of genotype on entry, e.g. from
 *   dock_score_batch), bias [n][G], rho [n], counts int32 [n][2] (successes,
 *   failures in a row). Inputs: normals [iterations][n][G], scale [G].
 *   energy_log: NULL or [n][iterations][2], the trials' energies (NaN where
 *   the second trial was not needed).
 * A call of K iterations followed by one of L equals one call of K + L with
 * the concatenated draws, bit for bit. Errors: DOCK_EINVAL on NULL handles,
 * opts or arrays, n < 0, iterations < 0, opts->n_genes other than the
 * ligand's gene count, run lengths < 1, a variant other
 * than SHUFFLE or MFMA_F32, a ligand never uploaded, a grid set without the
 * ligand's type maps, or misaligned arrays.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t iterations;
    int32_t n_genes;             /* G of the arrays; must equal the ligand's 7 + T */
    int32_t n_success;           /* successes in a row that double rho (AutoDock: 4) */
    int32_t n_failure;           /* failures in a row that halve rho (AutoDock: 4) */
    int32_t variant;             /* DOCK_REDUCE_SHUFFLE or DOCK_REDUCE_MFMA_F32 */
} dock_sw_opts;

int32_t dock_solis_wets_batch(const dock_grids* grids, const dock_ligand* ligand, int32_t n,
                              float* genotype_dev, float* energy_dev, float* bias_dev,
                              float* rho_dev, int32_t* counts_dev, const float* normals_dev,
                              const float* scale_dev, const dock_sw_opts* opts,
                              float* energy_log_dev, void* stream);

/* ------------------------------------------------------------------------
 * One generation step of the genetic search of the LGA (Sec. 2.1: the GA
 * produces new genotypes that the local search then improves; a docking job
 * holds many independent LGA runs). The paper names no operator; these are
 * the standard AutoDock ones:
 *   elitism      child 0 of each run copies the run's best member unchanged
 *                (lowest energy, lowest index among equals, NaN as +inf);
 *   selection    every other child takes two parents, each the winner of a
 *                binary tournament between two candidate members: the fitter
 *                (lower energy, the first candidate on a tie, NaN as +inf)
 *                wins when the tournament draw is < p_tournament, else the
 *                other;
 *   crossover    when the crossover draw is < p_crossover, genes [lo, hi)
 *                come from the second parent (lo, hi = the smaller and the
 *                larger cut point), the rest from the first;
 *   mutation     gene g changes when its draw is < p_mutation, by adding its
 *                displacement (one float32 addition, no fused operation).
 * Every random number is an input, drawn by the caller, so the result is
 * exact (reproducible bit for bit). All arrays are device, float32 or int32,
 * row-major, caller-owned:
 *   genotypes  [n_runs][pop][n_genes]  the current population
 *   energies   [n_runs][pop]           its energies
 *   candidates [n_runs][pop][4]        tournament candidates of parent 1
 *                                      (0, 1) and parent 2 (2, 3), member
 *                                      indices within the run, clamped to
 *                                      [0, pop - 1]; 16-byte aligned
 *   coins      [n_runs][pop][3]        draws of tournament 1, tournament 2
 *                                      and the crossover
 *   cuts       [n_runs][pop][2]        crossover cut points, clamped to
 *                                      [0, n_genes]; 8-byte aligned
 *   mut_coin   [n_runs][pop][n_genes]  mutation draws
 *   mut_delta  [n_runs][pop][n_genes]  mutation displacements
 *   children   [n_runs][pop][n_genes]  written; must not overlap genotypes
 *   best       [n_runs]                written: index of each run's best
 *                                      member (also without elitism)
 * Entries of child 0 of a run with elitism read no draws. The call queues
 * two kernels on `stream` (the best member per run, then one thread per
 * child gene) and returns; no host synchronisation, no allocation.
 * Errors: DOCK_EINVAL on a NULL descriptor or pointer, sizes < 1, n_genes >
 * DOCK_MAX_GENES, more than 2^31 - 1 child genes, a NaN probability,
 * elitism not 0 or 1, misaligned candidates or cuts, or overlapping
 * genotypes and children.
 * ---------------------------------------------------------------------- */
typedef struct {
    const float* genotypes;
    const float* energies;
    const int32_t* candidates;
    const float* coins;
    const int32_t* cuts;
    const float* mut_coin;
    const float* mut_delta;
    float* children;
    int32_t* best;
    int32_t n_runs;
    int32_t pop;
    int32_t n_genes;
    float p_tournament;
    float p_crossover;
    float p_mutation;
    int32_t elitism;
} dock_ga_step_desc;

int32_t dock_ga_step(const dock_ga_step_desc* desc, void* stream);

/* ------------------------------------------------------------------------
 * Local search on a share of the population (Sec. 2.1: the LGA improves the
 * genotypes the GA makes by local search; AutoDock searches each child with
 * a probability, the local-search rate). The caller draws one uniform number
 * per row; the rows with a draw below the rate are gathered into a compact
 * state, searched, and scattered back (the search's best genotypes and
 * energies replace the rows: Lamarckian write-back).
 *
 * dock_select_rows: index_dev[k] = the k-th row r, in increasing order, with
 * draws_dev[r] < rate (float32 comparison); *count_dev = the number of such
 * rows. draws_dev [n] float32, index_dev [n] int32 (entries past the count
 * are left as they were), count_dev [1] int32, device. One block of 1024
 * threads; deterministic. Errors: DOCK_EINVAL on n < 0, NULL arrays, a NaN
 * rate or misaligned arrays.
 * ---------------------------------------------------------------------- */
int32_t dock_select_rows(const float* draws_dev, int32_t n, float rate, int32_t* index_dev,
                         int32_t* count_dev, void* stream);

/* dock_gather_rows: dst_dev[k][c] = src_dev[index_dev[k]][c] for k < m and
 * c < row_floats; src_dev [n_src][row_floats], dst_dev [m][row_floats]
 * float32, index_dev [m] int32, device. Rows whose index lies outside
 * [0, n_src) are left unwritten.
 * dock_scatter_rows: dst_dev[index_dev[k]][c] = src_dev[k][c]; src_dev
 * [m][row_floats], dst_dev [n_dst][row_floats]; indices outside [0, n_dst)
 * are skipped; indices must be distinct (else the last write of a row is
 * unspecified). One thread per element. m == 0 is a no-op. Errors:
 * DOCK_EINVAL on negative sizes, row_floats < 1, more than 2^31 - 1
 * elements, NULL or misaligned arrays. */
int32_t dock_gather_rows(const float* src_dev, int32_t n_src, int32_t row_floats, const int32_t* index_dev,
                         int32_t m, float* dst_dev, void* stream);
int32_t dock_scatter_rows(const float* src_dev, int32_t m, int32_t row_floats, const int32_t* index_dev,
                          int32_t n_dst, float* dst_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DOCK_H */
