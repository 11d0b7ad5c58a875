// C ABI of the docking hot path (declarations and contracts in include/dock.h).
//
// Host-side responsibilities: argument validation before any device work,
// ligand preparation (dock_prep.cpp), the device item table of a local-search
// batch (staged through pinned host buffers and copied into the caller's
// workspace on the caller's stream), work ordering (longest items first) and
// launch geometry. Every compute step runs in the kernels of
// dock_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dock.h"
#include "dock_blob.h"
#include "dock_launch.h"
#include "dock_prep.h"

struct dock_grids {
    dock_grid_desc desc;
    docklaunch::GridParams gp;
};

struct dock_ligand {
    dockprep::Prepared prep;
    const uint8_t* blob_dev = nullptr;
    int slots = 1;
};

namespace {

thread_local std::string g_err;

int32_t fail(int32_t status, const std::string& msg) {
    g_err = msg;
    return status;
}

int32_t ok() { return DOCK_OK; }

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int32_t hip_fail(hipError_t e, const char* what) {
    return fail(DOCK_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Pinned staging buffers for host -> device copies of item tables. A buffer
// is reused only after the copy that last read it has executed (event).
class StagingRing {
  public:
    int32_t copy_to_device(void* dst, const void* src, size_t bytes, hipStream_t stream) {
        std::lock_guard<std::mutex> lock(mu_);
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        auto& ring = rings_[dev];
        Slot& s = ring.slot[ring.next];
        ring.next = (ring.next + 1) % kSlots;
        if (s.ev) {
            e = hipEventSynchronize(s.ev);
            if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        } else {
            e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
            if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        }
        if (s.cap < bytes) {
            if (s.host) (void)hipHostFree(s.host);
            s.host = nullptr;
            s.cap = 0;
            size_t cap = std::max<size_t>(bytes, 4096);
            e = hipHostMalloc(&s.host, cap, hipHostMallocDefault);
            if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
            s.cap = cap;
        }
        std::memcpy(s.host, src, bytes);
        e = hipMemcpyAsync(dst, s.host, bytes, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
        e = hipEventRecord(s.ev, stream);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        return DOCK_OK;
    }

  private:
    static constexpr int kSlots = 8;
    struct Slot {
        void* host = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
    };
    struct Ring {
        Slot slot[kSlots];
        int next = 0;
    };
    std::mutex mu_;
    std::map<int, Ring> rings_;
};

StagingRing& staging() {
    static StagingRing* r = new StagingRing();  // never destroyed: outlives late stream work
    return *r;
}

int device_cu_count(int32_t& out) {
    static std::mutex mu;
    static int cache[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(mu);
    if (dev < 0 || dev >= 64 || cache[dev] == 0) {
        int n = 0;
        e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
        if (dev >= 0 && dev < 64) cache[dev] = n;
        out = n;
        return DOCK_OK;
    }
    out = cache[dev];
    return DOCK_OK;
}

// Library-owned streams per device, used to run the second and later
// persistent launches of a split batch beside the first: they are forked
// from the caller's stream with an event and joined back into it with
// others, so the caller's later work still waits for all of them. The
// fork-launch-join sequence is serialised, since the events are shared.
constexpr int kLsFamilies = 5;
static_assert(8 + kLsFamilies <= docklaunch::kWorkspaceHeader / 4, "work counters fit the workspace header");
struct SideStream {
    hipStream_t stream[kLsFamilies - 1] = {};
    hipEvent_t fork = nullptr, join[kLsFamilies - 1] = {};
};

int side_stream(SideStream*& out, std::unique_lock<std::mutex>& lock) {
    static std::mutex mu;
    static std::map<int, SideStream>* table = new std::map<int, SideStream>();  // outlives late work
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    lock = std::unique_lock<std::mutex>(mu);
    SideStream& s = (*table)[dev];
    if (!s.stream[0]) {
        for (int k = 0; k < kLsFamilies - 1 && e == hipSuccess; ++k) {
            e = hipStreamCreateWithFlags(&s.stream[k], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&s.join[k], hipEventDisableTiming);
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.fork, hipEventDisableTiming);
        if (e != hipSuccess) {
            s = SideStream();
            return hip_fail(e, "side stream creation");
        }
    }
    out = &s;
    return DOCK_OK;
}

int32_t check_grid_for_ligand(const dock_grids* g, const dock_ligand* l) {
    if (l->prep.max_class >= g->desc.n_maps - 2)
        return fail(DOCK_EINVAL, "ligand uses an atom class with no type map in the grid set");
    return DOCK_OK;
}

bool valid_variant(int v) { return v >= 0 && v < DOCK_REDUCE_COUNT; }

// Storage of one call's plan; every array holds at least max(n_items, 1)
// entries, table kWorkspaceHeader + that many item records.
struct LsPlanBuf {
    docklaunch::DevItem* dev;
    int64_t* cost;
    int* fam;
    int* idx;
    uint8_t* table;
};

struct LsPart {
    int first, count, mode, variant;
    int64_t units, block_units;
    double block_work, wave_work;   // shared launch: estimated wave-slot time of either phase
};

struct LsPlan {
    LsPart part[kLsFamilies];
    int n_parts = 0;
    int64_t table_bytes = 0;
};

// Validates a local-search call and builds its device item table (header of
// zeroed work counters, then the items grouped by launch) in buf.table.
// n_parts = 0 when no item has work. Allocates nothing.
int32_t ls_plan(const dock_ls_item* items, int32_t n_items, const dock_ls_opts* o, LsPlanBuf& buf,
                LsPlan& plan) {
    plan = LsPlan();
    if (!o) return fail(DOCK_EINVAL, "dock_local_search_batch: NULL opts");
    if (n_items < 0 || (n_items > 0 && !items)) return fail(DOCK_EINVAL, "dock_local_search_batch: bad items");
    if (o->iterations < 0) return fail(DOCK_EINVAL, "iterations must be >= 0");
    if (!(o->rho > 0.f && o->rho < 1.f)) return fail(DOCK_EINVAL, "rho must be in (0, 1)");
    if (!(o->eps > 0.f) || !std::isfinite(o->eps)) return fail(DOCK_EINVAL, "eps must be > 0");
    if (!valid_variant(o->variant)) return fail(DOCK_EINVAL, "unknown default variant");
    if (o->threads_per_ind != 0 && o->threads_per_ind != 64 && o->threads_per_ind != 128 &&
        o->threads_per_ind != 256)
        return fail(DOCK_EUNSUPPORTED, "threads_per_ind must be 0, 64, 128 or 256");
    if ((o->flags & ~(DOCK_LS_FINAL_EVAL | DOCK_LS_SEPARATE_LAUNCHES)) != 0) return fail(DOCK_EINVAL, "unknown flags");
    docklaunch::DevItem* dev = buf.dev;
    int64_t* cost = buf.cost;
    // kernel family: 0 four waves, 1 two waves, 2 one wave with two atom
    // slots, 3 one wave with one slot, 4 two individuals per wave
    int* fam = buf.fam;
    int n_dev = 0;
    int64_t total = 0;
    bool any_fam[kLsFamilies] = {};
    bool any_plain = false;
    int var_u = -2;
    for (int i = 0; i < n_items; ++i) {
        const dock_ls_item& it = items[i];
        if (!it.grids || !it.ligand) return fail(DOCK_EINVAL, "item " + std::to_string(i) + ": NULL handle");
        if (it.n_genes != 7 + it.ligand->prep.n_torsions)
            return fail(DOCK_EINVAL, "item " + std::to_string(i) + ": n_genes " + std::to_string(it.n_genes) +
                                         " is not the ligand's " + std::to_string(7 + it.ligand->prep.n_torsions));
        if (it.n < 0) return fail(DOCK_EINVAL, "item " + std::to_string(i) + ": n < 0");
        int32_t st = check_grid_for_ligand(it.grids, it.ligand);
        if (st != DOCK_OK) return st;
        const int var = it.variant < 0 ? o->variant : it.variant;
        if (!valid_variant(var)) return fail(DOCK_EINVAL, "item " + std::to_string(i) + ": unknown variant");
        if (it.iterations < -1 || it.iterations > o->iterations)
            return fail(DOCK_EINVAL, "item " + std::to_string(i) + ": iterations outside [-1, opts->iterations]");
        if (it.final_eval < -1 || it.final_eval > 1)
            return fail(DOCK_EINVAL, "item " + std::to_string(i) + ": final_eval must be -1, 0 or 1");
        if (it.threads_per_ind != 0 && it.threads_per_ind != 64 && it.threads_per_ind != 128 &&
            it.threads_per_ind != 256)
            return fail(DOCK_EINVAL, "item " + std::to_string(i) + ": threads_per_ind must be 0, 64, 128 or 256");
        const int tpi = it.threads_per_ind != 0 ? it.threads_per_ind
                                                : (o->threads_per_ind != 0 ? o->threads_per_ind : 64);
        const int iters = it.iterations < 0 ? o->iterations : it.iterations;
        const int fin = it.final_eval < 0 ? ((o->flags & DOCK_LS_FINAL_EVAL) ? 1 : 0) : it.final_eval;
        if ((it.flags & ~(DOCK_ITEM_PLAIN_MAPS | DOCK_ITEM_TWO_PER_WAVE)) != 0)
            return fail(DOCK_EINVAL, "item " + std::to_string(i) + ": unknown flags");
        const bool two = (it.flags & DOCK_ITEM_TWO_PER_WAVE) != 0;
        if (two && (it.ligand->prep.n_atoms > 32 || it.n_genes > 32 || var != DOCK_REDUCE_SHUFFLE || tpi != 64))
            return fail(DOCK_EUNSUPPORTED, "item " + std::to_string(i) + ": two individuals per wave need <= 32 atoms, "
                                           "<= 32 genes, the shuffle reduction and 64 threads per individual");
        if (!it.ligand->blob_dev) return fail(DOCK_EINVAL, "item " + std::to_string(i) + ": ligand not uploaded");
        if (it.n == 0) continue;
        void* ptrs[] = {it.genotype, it.acc_g2, it.acc_dx2, it.best_genotype, it.best_energy, it.energy,
                        it.iters_done};
        for (void* p : ptrs)
            if (!p || !aligned(p, 4)) return fail(DOCK_EINVAL, "item " + std::to_string(i) + ": NULL or misaligned state");
        if (it.grad && !aligned(it.grad, 4)) return fail(DOCK_EINVAL, "item " + std::to_string(i) + ": misaligned grad");
        if (iters == 0 && !fin) continue;  // nothing to do for this item
        docklaunch::DevItem& d = dev[n_dev];
        std::memset(&d, 0, sizeof(d));
        d.grid = it.grids->gp;
        if (it.flags & DOCK_ITEM_PLAIN_MAPS) d.grid.corners = nullptr;
        any_plain = any_plain || d.grid.corners == nullptr;
        d.blob = it.ligand->blob_dev;
        d.genotype = it.genotype;
        d.acc_g2 = it.acc_g2;
        d.acc_dx2 = it.acc_dx2;
        d.best_genotype = it.best_genotype;
        d.best_energy = it.best_energy;
        d.energy = it.energy;
        d.iters_done = it.iters_done;
        d.grad = it.grad;
        d.n = it.n;
        d.variant = var;
        d.slots = it.ligand->slots;
        d.iterations = iters;
        d.final_eval = fin;
        d.pack = two ? 2 : 1;
        const auto& P = it.ligand->prep;
        const auto* H = reinterpret_cast<const dockblob::Header*>(P.blob.data());
        // per-individual cost: evaluations x (instruction estimate per
        // evaluation: pair batches, atom slots, torsion depth, fixed part)
        cost[n_dev] = (int64_t)(iters + fin) *
                      ((int64_t)H->n_batches * 90 + (int64_t)d.slots * (150 + 20 * P.max_depth) + 500);
        const int f = two ? 4 : (tpi == 256 ? 0 : (tpi == 128 ? 1 : (d.slots == 1 ? 3 : 2)));
        fam[n_dev] = f;
        any_fam[f] = true;
        var_u = (var_u == -2 || var_u == var) ? var : -1;
        total += it.n;
        ++n_dev;
    }
    if (total > 2147483647LL) return fail(DOCK_EUNSUPPORTED, "more than 2^31 individuals in one call");
    if (n_dev == 0) return ok();
    // A launch carries one kernel family, or one of two mixes that share a
    // launch when every item uses the same reduction variant: two-wave,
    // one-slot and two-per-wave items on corner-expanded maps (one launch of
    // 128-thread blocks, two-wave items first), or the two one-wave families
    // (the kernel dispatching on the atom layout per item). Otherwise, or on
    // request, there is one persistent launch per family (each with its own
    // work counter), in family order (four-wave items first, which have the
    // longest individuals), each group longest first. Carrying every
    // combination in one kernel would spill registers.
    const int var_uniform = var_u >= 0 ? var_u : -1;
    const bool shared_ok = var_uniform >= 0 && !(o->flags & DOCK_LS_SEPARATE_LAUNCHES);
    const int n_fams = (int)any_fam[0] + any_fam[1] + any_fam[2] + any_fam[3] + any_fam[4];
    const bool unified = shared_ok && n_fams >= 2 && !any_fam[0] && !any_fam[2] && !any_plain;
    const bool merge_one_wave = shared_ok && n_fams == 2 && any_fam[2] && any_fam[3];
    // unified: one part, two-wave items (group 0) before the one-wave units
    auto group = [&](int i) { return unified ? (fam[i] == 1 ? 0 : 1) : (merge_one_wave ? 2 : fam[i]); };
    auto part_of = [&](int i) { return unified ? 0 : group(i); };
    int* idx = buf.idx;
    for (int i = 0; i < n_dev; ++i) idx[i] = i;
    std::stable_sort(idx, idx + n_dev, [&](int a, int b) {
        if (group(a) != group(b)) return group(a) < group(b);
        return cost[a] > cost[b];
    });
    plan.table_bytes = docklaunch::kWorkspaceHeader + (int64_t)n_dev * (int64_t)sizeof(docklaunch::DevItem);
    std::memset(buf.table, 0, (size_t)plan.table_bytes);
    docklaunch::DevItem* tab = reinterpret_cast<docklaunch::DevItem*>(buf.table + docklaunch::kWorkspaceHeader);
    int32_t ub = 0;
    for (int i = 0; i < n_dev; ++i) {
        const int g = group(idx[i]);
        if (i == 0 || part_of(idx[i]) != part_of(idx[i - 1])) {
            static constexpr int kModes[kLsFamilies] = {docklaunch::kFourWave, docklaunch::kTwoWave,
                                                        docklaunch::kSlots2, docklaunch::kSlots1,
                                                        docklaunch::kTwoPerWave};
            const int mode = unified ? docklaunch::kUnified
                                     : (merge_one_wave ? docklaunch::kSlotsAny : kModes[g]);
            plan.part[plan.n_parts++] = {i, 0, mode, -1, 0, 0, 0.0, 0.0};
            ub = 0;
        }
        tab[i] = dev[idx[i]];
        tab[i].unit_begin = ub;
        // work units: individuals, or pairs of individuals two to a wave
        const int units = tab[i].pack == 2 ? (tab[i].n + 1) / 2 : tab[i].n;
        ub += units;
        plan.part[plan.n_parts - 1].units += units;
        if (unified) {
            // wave-slot time: two waves per individual take about 0.6 of one
            // wave's time on two slots; two per wave about 1.3 of it for two
            LsPart& pt = plan.part[plan.n_parts - 1];
            const double work = (double)cost[idx[i]] * tab[i].n;
            if (fam[idx[i]] == 1) {
                pt.block_units += units;
                pt.block_work += 1.25 * work;
            } else {
                pt.wave_work += (tab[i].pack == 2 ? 0.65 : 1.0) * work;
            }
        }
        ++plan.part[plan.n_parts - 1].count;
    }
    // each launch runs the kernel specialised for its items' variant when
    // they share one (e.g. a tuning table that picks one per size bucket)
    // (the specialised kernels read corner-expanded grids only; a part with an
    // item on plain maps runs the dispatching kernel, which reads either)
    for (int k = 0; k < plan.n_parts; ++k) {
        LsPart& pt = plan.part[k];
        int v = -2;
        bool corners = true;
        for (int i = pt.first; i < pt.first + pt.count; ++i) {
            v = (v == -2 || v == tab[i].variant) ? tab[i].variant : -1;
            corners = corners && tab[i].grid.corners != nullptr;
        }
        pt.variant = (v < 0 || !corners) ? -1 : v;
    }
    return ok();
}

// Blocks of a shared launch that skip the two-wave phase: the one-wave
// units' share of the estimated work, of the grid, so that both kinds of
// unit start at once (blocks that run out of two-wave units then turn to
// one-wave units). On the uneven 64-ligand batch this share made the launch
// 2-3 % faster than with every block starting on two-wave units, and than
// one launch per family; 1.25-1.5 times it gave less, twice it a slower
// launch.
constexpr double kSharedWaveShare = 1.0;

int shared_wave_blocks(const LsPart& pt, int grid) {
    const double total = pt.block_work + pt.wave_work;
    if (pt.block_units == 0) return grid;
    if (total <= 0.0) return 0;
    const int w = (int)(kSharedWaveShare * grid * pt.wave_work / total);
    return std::max(0, std::min(grid, w));
}

// Launches the parts of a plan whose table is already on its way to `ws`
// on `stream`. With side streams the second and later parts run beside the
// first on library-owned streams (forked from and joined back into
// `stream`); without, every part runs on `stream`, one after another.
int32_t ls_launch(const LsPlan& plan, const LsPlanBuf& buf, void* ws, const dock_ls_opts* o,
                  hipStream_t stream, bool side_streams) {
    const docklaunch::DevItem* tab =
        reinterpret_cast<const docklaunch::DevItem*>(buf.table + docklaunch::kWorkspaceHeader);
    int32_t n_cu = 0;
    int32_t st = device_cu_count(n_cu);
    if (st != DOCK_OK) return st;
    SideStream* side = nullptr;
    std::unique_lock<std::mutex> side_lock;
    const int n_side = side_streams ? plan.n_parts - 1 : 0;   // at most kLsFamilies - 1
    if (n_side > 0) {
        st = side_stream(side, side_lock);
        if (st != DOCK_OK) return st;
        hipError_t e = hipEventRecord(side->fork, stream);
        for (int k = 0; k < n_side && e == hipSuccess; ++k) e = hipStreamWaitEvent(side->stream[k], side->fork, 0);
        if (e != hipSuccess) return hip_fail(e, "dock_local_search_batch fork");
    }
    hipError_t launch_err = hipSuccess;
    for (int k = 0; k < plan.n_parts; ++k) {
        const LsPart& pt = plan.part[k];
        if (pt.count == 0) continue;
        const int64_t units = pt.units;
        int per_cu = docklaunch::ls_blocks_per_cu(pt.mode, pt.variant);
        if (per_cu <= 0) per_cu = 8;
        const int64_t resident = (int64_t)per_cu * n_cu;
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(units, resident));
        docklaunch::LsParams p;
        p.items = reinterpret_cast<const docklaunch::DevItem*>(static_cast<uint8_t*>(ws) +
                                                               docklaunch::kWorkspaceHeader) + pt.first;
        p.counter = static_cast<int32_t*>(ws) + k;
        p.n_items = pt.count;
        p.total_units = (int32_t)units;
        p.block_units = (int32_t)pt.block_units;
        p.counter2 = static_cast<int32_t*>(ws) + 8 + k;
        p.wave_blocks = pt.mode == docklaunch::kUnified ? shared_wave_blocks(pt, grid) : 0;
        p.rho = o->rho;
        p.eps = o->eps;
        hipStream_t s_k = (k == 0 || !side) ? stream : side->stream[k - 1];
        launch_err = docklaunch::launch_ls(p, pt.mode, pt.variant, grid, s_k);
        if (launch_err != hipSuccess) break;
    }
    if (side) {  // joined also after a failed launch
        hipError_t e = hipSuccess;
        for (int k = 0; k < n_side && e == hipSuccess; ++k) {
            e = hipEventRecord(side->join[k], side->stream[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(stream, side->join[k], 0);
        }
        if (e != hipSuccess && launch_err == hipSuccess) return hip_fail(e, "dock_local_search_batch join");
    }
    if (launch_err != hipSuccess) return hip_fail(launch_err, "dock_local_search_batch launch");
    return ok();
}


}  // namespace

extern "C" {

int32_t dock_abi_version(void) { return DOCK_ABI_VERSION; }

const char* dock_last_error(void) { return g_err.c_str(); }

int32_t dock_create_grids(const dock_grid_desc* d, const float* maps_dev, dock_grids** out) {
    if (!d || !maps_dev || !out) return fail(DOCK_EINVAL, "dock_create_grids: NULL argument");
    if (d->nx < 2 || d->ny < 2 || d->nz < 2) return fail(DOCK_EINVAL, "grid needs >= 2 nodes per axis");
    if (d->n_maps < 3) return fail(DOCK_EINVAL, "grid needs >= 3 maps (types, electrostatic, desolvation)");
    if (!(d->spacing > 0.f) || !std::isfinite(d->spacing)) return fail(DOCK_EINVAL, "grid spacing must be > 0");
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(d->origin[c])) return fail(DOCK_EINVAL, "grid origin must be finite");
    const double nodes = double(d->nx) * d->ny * d->nz * d->n_maps;
    if (nodes > 2147483647.0) return fail(DOCK_EUNSUPPORTED, "grid set exceeds 2^31 floats");
    if (!aligned(maps_dev, 4)) return fail(DOCK_EINVAL, "maps pointer not 4-byte aligned");
    dock_grids* g = new (std::nothrow) dock_grids();
    if (!g) return fail(DOCK_ENOMEM, "out of host memory");
    g->desc = *d;
    g->gp.maps = maps_dev;
    g->gp.corners = nullptr;
    g->gp.nx = d->nx;
    g->gp.ny = d->ny;
    g->gp.nz = d->nz;
    g->gp.n_maps = d->n_maps;
    g->gp.spacing = d->spacing;
    g->gp.inv_spacing = (float)(1.0 / (double)d->spacing);
    const int n[3] = {d->nx, d->ny, d->nz};
    for (int c = 0; c < 3; ++c) {
        g->gp.origin[c] = d->origin[c];
        g->gp.hi[c] = (float)((double)d->origin[c] + (double)(n[c] - 1) * (double)d->spacing);
    }
    *out = g;
    return ok();
}

int32_t dock_destroy_grids(dock_grids* g) {
    delete g;
    return ok();
}

int32_t dock_grids_corner_bytes(const dock_grids* g, int64_t* bytes) {
    if (!g || !bytes) return fail(DOCK_EINVAL, "dock_grids_corner_bytes: NULL argument");
    *bytes = (int64_t)(g->desc.n_maps - 2) * (g->desc.nx - 1) * (g->desc.ny - 1) * (g->desc.nz - 1) * 128;
    return ok();
}

int32_t dock_grids_bind_corners(dock_grids* g, void* corners_dev, int64_t bytes, void* stream) {
    if (!g) return fail(DOCK_EINVAL, "dock_grids_bind_corners: NULL grids");
    if (!corners_dev) {
        g->gp.corners = nullptr;
        return ok();
    }
    int64_t need = 0;
    dock_grids_corner_bytes(g, &need);
    if (bytes < need) return fail(DOCK_EINVAL, "corner buffer too small");
    if (!aligned(corners_dev, 16)) return fail(DOCK_EINVAL, "corner buffer must be 16-byte aligned");
    hipError_t e = docklaunch::launch_expand_corners(g->gp, static_cast<float*>(corners_dev),
                                                     (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "dock_grids_bind_corners launch");
    g->gp.corners = static_cast<const float*>(corners_dev);
    return ok();
}

int32_t dock_create_ligand(const dock_ligand_desc* d, dock_ligand** out) {
    if (!d || !out) return fail(DOCK_EINVAL, "dock_create_ligand: NULL argument");
    dock_ligand* l = new (std::nothrow) dock_ligand();
    if (!l) return fail(DOCK_ENOMEM, "out of host memory");
    std::string err;
    int32_t st;
    try {
        st = dockprep::prepare(*d, l->prep, err);
    } catch (const std::bad_alloc&) {
        delete l;
        return fail(DOCK_ENOMEM, "out of host memory");
    }
    if (st != DOCK_OK) {
        delete l;
        return fail(st, "dock_create_ligand: " + err);
    }
    l->slots = l->prep.n_atoms <= 64 ? 1 : 2;
    *out = l;
    return ok();
}

int32_t dock_ligand_info_get(const dock_ligand* l, dock_ligand_info* out) {
    if (!l || !out) return fail(DOCK_EINVAL, "dock_ligand_info_get: NULL argument");
    out->n_atoms = l->prep.n_atoms;
    out->n_torsions = l->prep.n_torsions;
    out->n_genes = 7 + l->prep.n_torsions;
    out->n_pairs = l->prep.n_pairs;
    out->n_fragments = l->prep.n_frag;
    out->max_depth = l->prep.max_depth;
    {
        const dockblob::Header* h = reinterpret_cast<const dockblob::Header*>(l->prep.blob.data());
        out->n_batches = h->n_batches;
        out->n_copies = h->n_copies;
    }
    out->blob_bytes = (int64_t)l->prep.blob.size();
    return ok();
}

int32_t dock_ligand_export(const dock_ligand* l, int32_t* order, int32_t* torsions, int32_t* fragment,
                           uint32_t* pairs, uint8_t* pair_hb, uint32_t* batches) {
    if (!l) return fail(DOCK_EINVAL, "dock_ligand_export: NULL ligand");
    const auto& P = l->prep;
    if (order) std::copy(P.order.begin(), P.order.end(), order);
    if (torsions)
        for (int k = 0; k < P.n_torsions; ++k) {
            torsions[4 * k + 0] = P.tors_a[k];
            torsions[4 * k + 1] = P.tors_b[k];
            torsions[4 * k + 2] = P.tors_first[k];
            torsions[4 * k + 3] = P.tors_end[k];
        }
    if (fragment) std::copy(P.frag_of_atom.begin(), P.frag_of_atom.end(), fragment);
    if (pairs || pair_hb) {
        std::vector<uint32_t> pv;
        std::vector<uint8_t> hv;
        dockprep::decode_pairs(P, pv, hv);
        if (pairs) std::copy(pv.begin(), pv.end(), pairs);
        if (pair_hb) std::copy(hv.begin(), hv.end(), pair_hb);
    }
    if (batches) {
        const dockblob::Header* h = reinterpret_cast<const dockblob::Header*>(P.blob.data());
        for (int k = 0; k < h->n_batches * dockblob::kBatch; ++k) batches[k] = dockprep::record_of(P, k);
    }
    return ok();
}

int32_t dock_ligand_upload(dock_ligand* l, void* blob_dev, void* stream) {
    if (!l || !blob_dev) return fail(DOCK_EINVAL, "dock_ligand_upload: NULL argument");
    if (!aligned(blob_dev, 16)) return fail(DOCK_EINVAL, "ligand blob must be 16-byte aligned");
    // staged through pinned memory: asynchronous on the stream, no host wait
    int32_t st = staging().copy_to_device(blob_dev, l->prep.blob.data(), l->prep.blob.size(),
                                          (hipStream_t)stream);
    if (st != DOCK_OK) return st;
    l->blob_dev = static_cast<const uint8_t*>(blob_dev);
    return ok();
}

int32_t dock_destroy_ligand(dock_ligand* l) {
    delete l;
    return ok();
}

int32_t dock_score_batch(const dock_grids* g, const dock_ligand* l, int32_t n, const float* gen,
                         float* energy, float* grad, const dock_exec_opts* o, void* stream) {
    if (!g || !l) return fail(DOCK_EINVAL, "dock_score_batch: NULL handle");
    if (n < 0) return fail(DOCK_EINVAL, "dock_score_batch: n < 0");
    if (!l->blob_dev) return fail(DOCK_EINVAL, "dock_score_batch: ligand not uploaded");
    int32_t st = check_grid_for_ligand(g, l);
    if (st != DOCK_OK) return st;
    const int variant = o ? o->variant : DOCK_REDUCE_SHUFFLE;
    if (!valid_variant(variant)) return fail(DOCK_EINVAL, "dock_score_batch: unknown variant");
    if (o && o->threads_per_ind != 0 && o->threads_per_ind != 64)
        return fail(DOCK_EUNSUPPORTED, "dock_score_batch: threads_per_ind must be 0 or 64");
    if (o && (o->flags & ~DOCK_EXEC_TWO_PER_WAVE) != 0) return fail(DOCK_EINVAL, "dock_score_batch: unknown flags");
    const bool two = o && (o->flags & DOCK_EXEC_TWO_PER_WAVE);
    if (two && (l->prep.n_atoms > 32 || 7 + l->prep.n_torsions > 32 || variant != DOCK_REDUCE_SHUFFLE))
        return fail(DOCK_EUNSUPPORTED, "dock_score_batch: two genotypes per wave need <= 32 atoms, <= 32 genes "
                                       "and the shuffle reduction");
    if (n == 0) return ok();
    if (!gen || !energy) return fail(DOCK_EINVAL, "dock_score_batch: NULL genotypes or energy");
    if (!aligned(gen, 4) || !aligned(energy, 4) || (grad && !aligned(grad, 4)))
        return fail(DOCK_EINVAL, "dock_score_batch: pointers must be 4-byte aligned");
    float* atom_out = o ? o->atom_out : nullptr;
    if (atom_out && !aligned(atom_out, 16)) return fail(DOCK_EINVAL, "atom_out must be 16-byte aligned");
    int32_t n_cu = 0;
    st = device_cu_count(n_cu);
    if (st != DOCK_OK) return st;
    hipError_t e = two ? docklaunch::launch_score_two(g->gp, l->blob_dev, n, gen, energy, grad, atom_out, n_cu,
                                                      (hipStream_t)stream)
                       : docklaunch::launch_score(g->gp, l->blob_dev, l->slots, n, gen, energy, grad, atom_out,
                                                  variant, n_cu, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "dock_score_batch launch");
    return ok();
}

int32_t dock_ls_workspace_bytes(int32_t n_items, int64_t* bytes) {
    if (n_items < 0 || !bytes) return fail(DOCK_EINVAL, "dock_ls_workspace_bytes: bad argument");
    *bytes = docklaunch::kWorkspaceHeader + (int64_t)n_items * (int64_t)sizeof(docklaunch::DevItem);
    return ok();
}

int32_t dock_local_search_batch(const dock_ls_item* items, int32_t n_items, const dock_ls_opts* o,
                                void* ws, int64_t ws_bytes, void* stream) {
    if (n_items < 0 || (n_items > 0 && !items)) return fail(DOCK_EINVAL, "dock_local_search_batch: bad items");
    std::vector<docklaunch::DevItem> dev(std::max(n_items, 1));
    std::vector<int64_t> cost(std::max(n_items, 1));
    std::vector<int> fam(std::max(n_items, 1)), idx(std::max(n_items, 1));
    std::vector<uint8_t> table(docklaunch::kWorkspaceHeader + (size_t)std::max(n_items, 1) * sizeof(docklaunch::DevItem));
    LsPlanBuf buf{dev.data(), cost.data(), fam.data(), idx.data(), table.data()};
    LsPlan plan;
    int32_t st = ls_plan(items, n_items, o, buf, plan);
    if (st != DOCK_OK || plan.n_parts == 0) return st;
    int64_t need = 0;
    dock_ls_workspace_bytes(n_items, &need);
    if (!ws) return fail(DOCK_EINVAL, "dock_local_search_batch: NULL workspace");
    if (ws_bytes < need) return fail(DOCK_EINVAL, "dock_local_search_batch: workspace too small");
    if (!aligned(ws, 16)) return fail(DOCK_EINVAL, "workspace must be 16-byte aligned");
    // counters (one 32-bit word per part in the header) start at 0: they are
    // part of the copy
    st = staging().copy_to_device(ws, table.data(), plan.table_bytes, (hipStream_t)stream);
    if (st != DOCK_OK) return st;
    return ls_launch(plan, buf, ws, o, (hipStream_t)stream, true);
}

int32_t dock_ls_launches(const dock_ls_item* items, int32_t n_items, const dock_ls_opts* o,
                         int32_t* n_launches) {
    if (!n_launches) return fail(DOCK_EINVAL, "dock_ls_launches: NULL n_launches");
    if (n_items < 0 || (n_items > 0 && !items)) return fail(DOCK_EINVAL, "dock_ls_launches: bad items");
    std::vector<docklaunch::DevItem> dev(std::max(n_items, 1));
    std::vector<int64_t> cost(std::max(n_items, 1));
    std::vector<int> fam(std::max(n_items, 1)), idx(std::max(n_items, 1));
    std::vector<uint8_t> table(docklaunch::kWorkspaceHeader + (size_t)std::max(n_items, 1) * sizeof(docklaunch::DevItem));
    LsPlanBuf buf{dev.data(), cost.data(), fam.data(), idx.data(), table.data()};
    LsPlan plan;
    const int32_t st = ls_plan(items, n_items, o, buf, plan);
    if (st != DOCK_OK) return st;
    *n_launches = plan.n_parts;
    return ok();
}

int32_t dock_local_search_batch_static(const dock_ls_item* items, int32_t n_items, const dock_ls_opts* o,
                                       void* stream) {
    if (n_items < 0 || (n_items > 0 && !items))
        return fail(DOCK_EINVAL, "dock_local_search_batch_static: bad items");
    if (n_items > DOCK_STATIC_MAX_ITEMS)
        return fail(DOCK_EINVAL, "dock_local_search_batch_static: " + std::to_string(n_items) +
                                     " items exceed DOCK_STATIC_MAX_ITEMS (" +
                                     std::to_string(DOCK_STATIC_MAX_ITEMS) + ")");
    docklaunch::DevItem dev[DOCK_STATIC_MAX_ITEMS];
    int64_t cost[DOCK_STATIC_MAX_ITEMS];
    int fam[DOCK_STATIC_MAX_ITEMS], idx[DOCK_STATIC_MAX_ITEMS];
    alignas(16) uint8_t table[docklaunch::kWorkspaceHeader + DOCK_STATIC_MAX_ITEMS * sizeof(docklaunch::DevItem)];
    LsPlanBuf buf{dev, cost, fam, idx, table};
    LsPlan plan;
    int32_t st = ls_plan(items, n_items, o, buf, plan);
    if (st != DOCK_OK || plan.n_parts == 0) return st;
    if (plan.table_bytes > docklaunch::static_workspace_capacity())
        return fail(DOCK_EINVAL, "dock_local_search_batch_static: item table exceeds the static workspace");
    void* ws = nullptr;
    hipError_t e = docklaunch::static_workspace(&ws);
    if (e != hipSuccess) return hip_fail(e, "dock_local_search_batch_static: workspace address");
    // the fill kernel writes the whole table, counters included (zeros)
    e = docklaunch::launch_table_fill(ws, table, plan.table_bytes, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "dock_local_search_batch_static: table fill");
    return ls_launch(plan, buf, ws, o, (hipStream_t)stream, false);
}

int32_t dock_block_sum4(const float* in, float* out, int32_t n_blocks, int32_t threads, int32_t variant,
                        int32_t repeat, void* stream) {
    if (!in || !out) return fail(DOCK_EINVAL, "dock_block_sum4: NULL pointer");
    if (n_blocks < 0 || threads < 64 || threads > 1024 || threads % 64 != 0 || repeat < 1)
        return fail(DOCK_EINVAL, "dock_block_sum4: bad sizes");
    if (variant < 0 || variant > DOCK_REDUCE_SHARED_ATOMIC) return fail(DOCK_EINVAL, "dock_block_sum4: unknown variant");
    if (!aligned(in, 16) || !aligned(out, 16)) return fail(DOCK_EINVAL, "dock_block_sum4: need 16-byte alignment");
    if (n_blocks == 0) return ok();
    hipError_t e = docklaunch::launch_block_sum4(in, out, n_blocks, threads, variant, repeat, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "dock_block_sum4 launch");
    return ok();
}

int32_t dock_solis_wets_batch(const dock_grids* g, const dock_ligand* l, int32_t n, float* genotype,
                              float* energy, float* bias, float* rho, int32_t* counts, const float* normals,
                              const float* scale, const dock_sw_opts* o, float* energy_log, void* stream) {
    if (!g || !l || !o) return fail(DOCK_EINVAL, "dock_solis_wets_batch: NULL handle or opts");
    if (n < 0 || o->iterations < 0) return fail(DOCK_EINVAL, "dock_solis_wets_batch: n or iterations < 0");
    if (o->n_success < 1 || o->n_failure < 1) return fail(DOCK_EINVAL, "dock_solis_wets_batch: run lengths must be >= 1");
    if (o->variant != DOCK_REDUCE_SHUFFLE && o->variant != DOCK_REDUCE_MFMA_F32)
        return fail(DOCK_EINVAL, "dock_solis_wets_batch: variant must be SHUFFLE or MFMA_F32");
    if (o->n_genes != 7 + l->prep.n_torsions)
        return fail(DOCK_EINVAL, "dock_solis_wets_batch: n_genes " + std::to_string(o->n_genes) +
                                     " is not the ligand's " + std::to_string(7 + l->prep.n_torsions));
    if (!l->blob_dev) return fail(DOCK_EINVAL, "dock_solis_wets_batch: ligand not uploaded");
    int32_t st = check_grid_for_ligand(g, l);
    if (st != DOCK_OK) return st;
    if (n == 0) return ok();
    if (!genotype || !energy || !bias || !rho || !counts || !scale || (o->iterations > 0 && !normals))
        return fail(DOCK_EINVAL, "dock_solis_wets_batch: NULL array");
    if (!aligned(genotype, 4) || !aligned(energy, 4) || !aligned(bias, 4) || !aligned(rho, 4) ||
        !aligned(counts, 4) || !aligned(scale, 4) || (normals && !aligned(normals, 4)) ||
        (energy_log && !aligned(energy_log, 4)))
        return fail(DOCK_EINVAL, "dock_solis_wets_batch: arrays must be 4-byte aligned");
    docklaunch::SwParams p;
    p.normals = normals;
    p.scale = scale;
    p.genotype = genotype;
    p.energy = energy;
    p.bias = bias;
    p.rho = rho;
    p.counts = counts;
    p.log = energy_log;
    p.n = n;
    p.iterations = o->iterations;
    p.n_success = o->n_success;
    p.n_failure = o->n_failure;
    hipError_t e = docklaunch::launch_sw(g->gp, l->blob_dev, l->slots, o->variant, p, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "dock_solis_wets_batch launch");
    return ok();
}

int32_t dock_ga_step(const dock_ga_step_desc* d, void* stream) {
    if (!d) return fail(DOCK_EINVAL, "dock_ga_step: NULL descriptor");
    if (!d->genotypes || !d->energies || !d->candidates || !d->coins || !d->cuts || !d->mut_coin ||
        !d->mut_delta || !d->children || !d->best)
        return fail(DOCK_EINVAL, "dock_ga_step: NULL pointer");
    if (d->n_runs < 1 || d->pop < 1 || d->n_genes < 1 || d->n_genes > DOCK_MAX_GENES)
        return fail(DOCK_EINVAL, "dock_ga_step: bad sizes");
    const int64_t genes = (int64_t)d->n_runs * d->pop * d->n_genes;
    if (genes > 2147483647LL) return fail(DOCK_EINVAL, "dock_ga_step: more than 2^31 - 1 child genes");
    if (std::isnan(d->p_tournament) || std::isnan(d->p_crossover) || std::isnan(d->p_mutation))
        return fail(DOCK_EINVAL, "dock_ga_step: NaN probability");
    if (d->elitism != 0 && d->elitism != 1) return fail(DOCK_EINVAL, "dock_ga_step: elitism must be 0 or 1");
    if (!aligned(d->candidates, 16) || !aligned(d->cuts, 8) || !aligned(d->genotypes, 4) ||
        !aligned(d->energies, 4) || !aligned(d->coins, 4) || !aligned(d->mut_coin, 4) ||
        !aligned(d->mut_delta, 4) || !aligned(d->children, 4) || !aligned(d->best, 4))
        return fail(DOCK_EINVAL, "dock_ga_step: misaligned array");
    const uintptr_t g0 = reinterpret_cast<uintptr_t>(d->genotypes), c0 = reinterpret_cast<uintptr_t>(d->children);
    const uintptr_t span = (uintptr_t)genes * sizeof(float);
    if (g0 < c0 + span && c0 < g0 + span) return fail(DOCK_EINVAL, "dock_ga_step: children overlap genotypes");
    docklaunch::GaParams p;
    p.genotypes = d->genotypes;
    p.energies = d->energies;
    p.cand = d->candidates;
    p.coins = d->coins;
    p.cuts = d->cuts;
    p.mut_coin = d->mut_coin;
    p.mut_delta = d->mut_delta;
    p.children = d->children;
    p.best = d->best;
    p.n_runs = d->n_runs;
    p.pop = d->pop;
    p.n_genes = d->n_genes;
    p.p_tournament = d->p_tournament;
    p.p_crossover = d->p_crossover;
    p.p_mutation = d->p_mutation;
    p.elitism = d->elitism;
    hipError_t e = docklaunch::launch_ga_step(p, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "dock_ga_step launch");
    return ok();
}

int32_t dock_select_rows(const float* draws, int32_t n, float rate, int32_t* index, int32_t* count,
                         void* stream) {
    if (n < 0) return fail(DOCK_EINVAL, "dock_select_rows: n < 0");
    if (!count) return fail(DOCK_EINVAL, "dock_select_rows: NULL count");
    if (n > 0 && (!draws || !index)) return fail(DOCK_EINVAL, "dock_select_rows: NULL draws or index");
    if (std::isnan(rate)) return fail(DOCK_EINVAL, "dock_select_rows: NaN rate");
    if (!aligned(count, 4) || (draws && !aligned(draws, 4)) || (index && !aligned(index, 4)))
        return fail(DOCK_EINVAL, "dock_select_rows: arrays must be 4-byte aligned");
    hipError_t e = docklaunch::launch_select_rows(draws, n, rate, index, count, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "dock_select_rows launch");
    return ok();
}

static int32_t move_rows(bool gather, const float* src, float* dst, const int32_t* index, int32_t m,
                         int32_t row, int32_t n_rows, void* stream, const char* name) {
    if (m < 0 || row < 1 || n_rows < 0) return fail(DOCK_EINVAL, std::string(name) + ": bad sizes");
    if ((long long)m * row > 2147483647LL || (long long)n_rows * row > 2147483647LL)
        return fail(DOCK_EINVAL, std::string(name) + ": more than 2^31 - 1 elements");
    if (m == 0) return ok();
    if (!src || !dst || !index) return fail(DOCK_EINVAL, std::string(name) + ": NULL pointer");
    if (!aligned(src, 4) || !aligned(dst, 4) || !aligned(index, 4))
        return fail(DOCK_EINVAL, std::string(name) + ": arrays must be 4-byte aligned");
    hipError_t e = docklaunch::launch_move_rows(gather, src, dst, index, m, row, n_rows, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, (std::string(name) + " launch").c_str());
    return ok();
}

int32_t dock_gather_rows(const float* src, int32_t n_src, int32_t row, const int32_t* index, int32_t m,
                         float* dst, void* stream) {
    return move_rows(true, src, dst, index, m, row, n_src, stream, "dock_gather_rows");
}

int32_t dock_scatter_rows(const float* src, int32_t m, int32_t row, const int32_t* index, int32_t n_dst,
                          float* dst, void* stream) {
    return move_rows(false, src, dst, index, m, row, n_dst, stream, "dock_scatter_rows");
}

}  // extern "C"
