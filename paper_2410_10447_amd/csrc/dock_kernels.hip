// HIP kernels of the docking hot path for gfx950 (MI355X, CDNA4, wave64).
//
// One wave owns one individual. The per-evaluation pipeline (Sec. 2.1 of the
// paper: pose from the genotype, pairwise free-energy terms, gradient and
// torque sums, ADADELTA step) runs entirely inside the wave:
//
//   genotype (lane c holds gene c)
//   -> torsion transforms (lane k: Rodrigues rotation about bond k)
//   -> atom positions (lane a: atom a in depth-first order, a second slot
//      holds atom a + 64 for ligands of 65..128 atoms): the torsions that
//      enclose the atom's fragment, innermost first, then the rigid rotation
//   -> grid term: trilinear interpolation of three maps per atom
//   -> pair terms: host-built batches of 64 kept pairs, one pair per lane,
//      forces added to per-copy LDS accumulators of both atoms
//   -> block sum of {E, gx, gy, gz} (Sec. 3/4.2; selectable shuffle or MFMA
//      variants); torque and torsion torques by a wave prefix scan
//   -> gradient with respect to the genotype, ADADELTA update.
//
// No barrier spans more than one wave, no LDS or global float atomics are
// used, and every sum runs in a fixed order, so results are deterministic
// run to run and independent of what else shares the launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "dock.h"
#include "dock_blob.h"
#include "dock_launch.h"

namespace {

using dockblob::Header;
using dockblob::Torsion;
using docklaunch::DevItem;
using docklaunch::GridParams;
using docklaunch::LsParams;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int kWave = 64;
// Fourth word of a raw buffer resource on CDNA (32-bit data format, no
// swizzle, no stride): loads address bytes [0, num_records).
constexpr int kBufferWord3 = 0x00020000;
constexpr int kMaxTors = dockblob::kMaxTorsions;
constexpr int kMaxFrag = dockblob::kMaxFrag;
constexpr int kChain = dockblob::kChainStride;

// Force-field constants (AutoDock4 forms, Mehler-Solmajer dielectric).
constexpr float kR2Min = 1.0e-4f;        // A^2 lower clamp on r^2
constexpr float kCap = 1.0e5f;           // cap of the 12-6 / 12-10 term
constexpr float kOut = 100.0f;           // outside-the-box penalty constant
constexpr float kDielA = -8.5525f;
constexpr float kDielB = 86.9525f;       // eps0 - A with eps0 = 78.4
constexpr float kDielK = 7.7839f;
constexpr float kDielLB = 0.003627f * 86.9525f;            // lambda * B
constexpr float kDielBKLB = 86.9525f * 7.7839f * 0.003627f * 86.9525f;
constexpr float kDsInv2S2 = 1.0f / (2.0f * 3.5f * 3.5f);   // 1 / (2 sigma^2)
constexpr float kDsInvS2 = 1.0f / (3.5f * 3.5f);
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kSqrtElec = 18.222613f;      // sqrt(332.06363 kcal A / (mol e^2)): charges in LDS carry it

// ---------------------------------------------------------------------------
// Cross-lane primitives (wave64).
// ---------------------------------------------------------------------------

template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ float dpp(float v) {
    // lanes whose source is outside the row, or whose row is masked off, read 0
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, BANK_MASK, true));
}

__device__ __forceinline__ float readlane(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Ordering of LDS accesses between the lanes of one wave, where one wave is
// everything that shares the data: a wave's LDS instructions execute in
// program order, so it only has to keep the compiler from moving LDS
// accesses across this point (a wavefront-scope fence orders them in the
// compiler; the wave barrier keeps the instruction scheduler from moving
// them). No block barrier: another wave of the block may be working on
// something else, at another point of its code.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// The LDS ordering an evaluation needs: the wave's own when it holds the
// whole individual, the block's when WAVES waves share it.
template <int WAVES>
__device__ __forceinline__ void lds_sync() {
    if constexpr (WAVES == 1) wave_sync();
    else __syncthreads();
}

// Wave-uniform value: lets the compiler keep it (and what is derived from it,
// such as loop bounds and addresses) in scalar registers.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

// Global-memory view of a pointer, so that loads are issued as global (not
// flat) instructions and do not count against the LDS wait counter.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p) {
    return (const __attribute__((address_space(1))) T*)(p);
}

// Sum over the wave, every lane receives the same value. Butterfly inside
// each 16-lane row with DPP (quad swaps, half-row and row mirrors), then the
// row sums S0..S3 are combined by row broadcasts as (S3 + S2) + (S1 + S0)
// in the last lane, which is read as a scalar.
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp<0xB1>(v);         // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);         // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);        // row_half_mirror
    v += dpp<0x140>(v);        // row_mirror
    v += dpp<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return readlane(v, 63);
}

__device__ __forceinline__ float wave_max(float v) {
    v = fmaxf(v, dpp<0xB1>(v));
    v = fmaxf(v, dpp<0x4E>(v));
    v = fmaxf(v, dpp<0x141>(v));
    v = fmaxf(v, dpp<0x140>(v));
    return fmaxf(fmaxf(readlane(v, 0), readlane(v, 16)), fmaxf(readlane(v, 32), readlane(v, 48)));
}

// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ float wave_scan(float v) {
    v += dpp<0x111>(v);          // row_shr:1
    v += dpp<0x112>(v);          // row_shr:2
    v += dpp<0x114>(v);          // row_shr:4
    v += dpp<0x118>(v);          // row_shr:8
    v += dpp<0x142, 0xa>(v);     // row_bcast:15 into rows 1 and 3
    v += dpp<0x143, 0xc>(v);     // row_bcast:31 into rows 2 and 3
    return v;
}

// ---------------------------------------------------------------------------
// Block sum of 4-vectors over one wave: the variants of the paper's step.
// ---------------------------------------------------------------------------

// R0: plain wavefront shuffle (the Sec. 3 baseline without its atomics and
// barriers: one wave needs neither).
__device__ __forceinline__ float4 sum4_shuffle(float4 v) {
    return make_float4(wave_sum(v.x), wave_sum(v.y), wave_sum(v.z), wave_sum(v.w));
}

// Tail shared by the MFMA variants. The 16x16 result holds, in column n,
// partial sums of component n % 4; lane l owns rows 4(l/16)..4(l/16)+3 of
// column l % 16. Adding its four rows and the matching lanes of the other
// three lane groups gives every lane the total of component l % 4.
__device__ __forceinline__ float4 mfma_tail(f32x4 acc) {
    float s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    return make_float4(readlane(s, 0), readlane(s, 1), readlane(s, 2), readlane(s, 3));
}

// R1: FP32 MFMA 16x16x4. The analogue of the paper's V = A P: each lane's
// component c enters A (row l % 16, k = l / 16); B is a 0/1 selection matrix
// that routes component c to the columns n with n % 4 == c, so four
// accumulating products leave, in each column, the sums over k (lanes l,
// l+16, l+32, l+48) of one component. The second product of the paper (Q V)
// is replaced by the in-register tail.
__device__ __forceinline__ float4 sum4_mfma_f32(float4 v) {
    const int c = lane_id() & 3;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v.x, c == 0 ? 1.f : 0.f, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v.y, c == 1 ? 1.f : 0.f, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v.z, c == 2 ? 1.f : 0.f, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v.w, c == 3 ? 1.f : 0.f, acc, 0, 0, 0);
    return mfma_tail(acc);
}

// R2: half-width MFMA 16x16x32 with split operands (precision refinement):
// each lane supplies 8 narrow values, hi and lo parts of its 4 components,
// B[k][n] = [k % 4 == n % 4], and the matrix unit adds hi + lo of 4 lanes per
// output element in FP32. The selection is invariant to how the unit maps
// (lane, slot) to k, since A and B share that mapping and k % 4 = slot % 4.
__device__ __forceinline__ bf16x8 sel_bf16() {
    const int c = lane_id() & 3;
    bf16x8 b;
#pragma unroll
    for (int i = 0; i < 8; ++i) b[i] = (__bf16)(((i & 3) == c) ? 1.0f : 0.0f);
    return b;
}

template <int TERMS>
__device__ __forceinline__ float4 sum4_mfma_bf16(float4 v) {
    const float vv[4] = {v.x, v.y, v.z, v.w};
    bf16x8 a;
    bf16x8 a2;
    float rem[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        __bf16 h = (__bf16)vv[i];
        a[i] = h;
        rem[i] = vv[i] - (float)h;
        __bf16 m = (__bf16)rem[i];
        a[4 + i] = m;
        rem[i] = rem[i] - (float)m;
        a2[i] = (__bf16)rem[i];
        a2[4 + i] = (__bf16)0.0f;
    }
    const bf16x8 b = sel_bf16();
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    if (TERMS == 3) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b, acc, 0, 0, 0);
    return mfma_tail(acc);
}

// FP16 has 5 exponent bits, so each component is first scaled by a power of
// two that brings the wave's largest magnitude just below 2^14 (exact), and
// the sum is scaled back (exact).
__device__ __forceinline__ float4 sum4_mfma_f16(float4 v) {
    const float vv[4] = {v.x, v.y, v.z, v.w};
    float mx[4] = {wave_max(fabsf(v.x)), wave_max(fabsf(v.y)), wave_max(fabsf(v.z)),
                   wave_max(fabsf(v.w))};
    int k[4];
    f16x8 a;
    f16x8 b;
    const int c = lane_id() & 3;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        k[i] = (mx[i] > 0.f && mx[i] <= 3.0e38f) ? 13 - ilogbf(mx[i]) : 0;
        k[i] = k[i] < -120 ? -120 : (k[i] > 120 ? 120 : k[i]);
        float s = ldexpf(vv[i], k[i]);
        _Float16 h = (_Float16)s;
        a[i] = h;
        a[4 + i] = (_Float16)(s - (float)h);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) b[i] = (_Float16)(((i & 3) == c) ? 1.0f : 0.0f);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc, 0, 0, 0);
    float4 t = mfma_tail(acc);
    return make_float4(ldexpf(t.x, -k[0]), ldexpf(t.y, -k[1]), ldexpf(t.z, -k[2]),
                       ldexpf(t.w, -k[3]));
}

template <int VAR>
__device__ __forceinline__ float4 sum4(float4 v) {
    if constexpr (VAR == DOCK_REDUCE_SHUFFLE) return sum4_shuffle(v);
    else if constexpr (VAR == DOCK_REDUCE_MFMA_F32) return sum4_mfma_f32(v);
    else if constexpr (VAR == DOCK_REDUCE_MFMA_BF16) return sum4_mfma_bf16<2>(v);
    else if constexpr (VAR == DOCK_REDUCE_MFMA_F16) return sum4_mfma_f16(v);
    else return sum4_mfma_bf16<3>(v);
}

// ---------------------------------------------------------------------------
// Ligand data held by a wave.
// ---------------------------------------------------------------------------

// LDS of one individual. Sized per layout: SLOTS atoms per lane and WAVES
// waves per individual (a wave of the two- and four-wave layouts owns 64
// atom positions, of which past the ligand's last atom none is used, and its
// own range of accumulator copies). A ligand of at most 64 atoms has at most
// 320 accumulator slots (n_copies * stride, n_copies <= 128/N + 2).
template <int SLOTS, int WAVES = 1>
struct __align__(16) Smem {
    static constexpr int kAtoms = kWave * SLOTS * WAVES;
    static constexpr int kSlots =
        (SLOTS == 1 && WAVES == 1) ? dockblob::kMaxSlotsSmall : dockblob::kMaxSlots * WAVES;
    float4 dyn[kAtoms];             // x, y, z relative to t, and sqrt(kElec) q (depth-first
                                    // order); zero past the last atom
    union {
        float tk[kMaxTors + 1][12]; // torsion transforms, 3x4 row-major, and the identity
                                    // (index kMaxTors); live until the atom positions are
                                    // written
        float4 acc[kSlots];         // pair-force accumulators, slot = (range * C + copy) *
                                    // stride + atom, one range per wave
    } u;
    float4 tor[kMaxTors][2];        // torsion k: axis point p and packed positions
                                    // (a | b << 8 | first << 16 | end << 24), unit axis u
    uint32_t chain[kMaxFrag][kChain / 4];  // per fragment: enclosing torsions, innermost
                                           // first, 4 per word, padded with the identity
    // several waves per individual: each wave's prefix sums of (g, x cross g)
    // at its atoms, and its {E, g} partial
    float pre[WAVES > 1 ? 6 : 1][WAVES > 1 ? kAtoms : 1];
    float4 xchg[WAVES][2];
    int unit;                       // several waves per individual: the block's work unit
};

template <int SLOTS>
struct Lig {
    // uniform
    int N, T, NF, G, n_batches, n_copies, max_depth;
    int stride;                     // accumulator stride (power of two >= N)
    int pmask;                      // stride * 16 - 1: slot byte offset -> position byte offset
    int wv;                         // wave of the individual (several waves per individual), else 0
    const u32x4* plist;             // pair records (dockblob::PairRec), n_batches x 64
    // per lane, per slot: atom a = lane + 64 * (slot + wv)
    float y0[SLOTS][3];
    float chg[SLOTS][3];            // 332.06363 q, q, |q|
    int cls[SLOTS];
    int frag[SLOTS];
    int orig[SLOTS];                // original atom index
};

template <int SLOTS, int WAVES = 1>
__device__ void load_ligand(const uint8_t* __restrict__ blob, Smem<SLOTS, WAVES>& sm, Lig<SLOTS>& L,
                            bool fill_lds = true) {
    if (fill_lds) lds_sync<WAVES>();  // previous users of the LDS tables are done
    const Header* h = reinterpret_cast<const Header*>(blob);
    const int lane = lane_id();
    L.wv = WAVES == 1 ? 0 : uniform((int)threadIdx.x >> 6);
    L.N = uniform(h->n_atoms);
    L.T = uniform(h->n_torsions);
    L.NF = uniform(h->n_frag);
    L.G = uniform(h->n_genes);
    L.n_batches = uniform(h->n_batches);
    L.n_copies = uniform(h->n_copies);
    L.max_depth = uniform(h->max_depth);
    L.stride = uniform(h->slot_stride);
    L.pmask = L.stride * 16 - 1;
    L.plist = uniform_ptr(reinterpret_cast<const u32x4*>(blob + h->off_plist));
    const float4* ref = reinterpret_cast<const float4*>(blob + h->off_ref);
    const float4* chg = reinterpret_cast<const float4*>(blob + h->off_chg);
    const int4* iv = reinterpret_cast<const int4*>(blob + h->off_int);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int a = lane + kWave * (s + L.wv);
        const bool ok = a < L.N;
        const int ai = ok ? a : 0;
        float4 r = ref[ai], c = chg[ai];
        int4 ii = iv[ai];
        L.y0[s][0] = r.x; L.y0[s][1] = r.y; L.y0[s][2] = r.z;
        L.chg[s][0] = ok ? c.x : 0.f; L.chg[s][1] = ok ? c.y : 0.f; L.chg[s][2] = ok ? c.z : 0.f;
        L.cls[s] = ii.x;
        L.frag[s] = ii.y;
        L.orig[s] = ii.z;
    }
    const Torsion* tr = reinterpret_cast<const Torsion*>(blob + h->off_tors);
    if (fill_lds && L.wv == 0 && lane < L.T) {
        const Torsion t = tr[lane];
        const int pk = t.a_pos | (t.b_pos << 8) | (t.first << 16) | (t.end << 24);
        sm.tor[lane][0] = make_float4(t.p[0], t.p[1], t.p[2], __int_as_float(pk));
        sm.tor[lane][1] = make_float4(t.u[0], t.u[1], t.u[2], 0.f);
    }
    const uint32_t* ch = reinterpret_cast<const uint32_t*>(blob + h->off_chain);
    const int n_chain_words = L.NF * (kChain / 4);
    uint32_t* dst = &sm.chain[0][0];
    if (fill_lds)
        for (int i = WAVES == 1 ? lane : (int)threadIdx.x; i < n_chain_words; i += kWave * WAVES) dst[i] = ch[i];
    lds_sync<WAVES>();
}

// ---------------------------------------------------------------------------
// Intermolecular grid term of one atom.
//
// The atom's world position is t + xl, with xl its position relative to the
// ligand's rotation centre. The cell is chosen from the rounded world
// coordinate, but the fraction inside the cell is taken from the exact
// difference to the cell's lower node, (t - node) + xl, summed with error
// compensation: a fraction derived from u = (x - origin)/h would carry the
// rounding of |u| (up to the grid size) into every interpolation weight.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float two_sum_fraction(float t, float node, float xl) {
    const float s = t - node;
    const float bp = s - t;
    const float e1 = (t - (s - bp)) + (-node - bp);
    const float s2 = s + xl;
    const float bq = s2 - s;
    const float e2 = (s - (s2 - bq)) + (xl - bq);
    return s2 + (e1 + e2);
}

// The fraction inside cell c (chosen when the loads were issued) along one
// axis, and the world and box-clamped coordinates.
__device__ __forceinline__ void axis_cell(float t, float xl, float lo, float hi, float h, float ih,
                                          int c, float& f, float& xw, float& xc) {
    xw = t + xl;
    xc = fminf(fmaxf(xw, lo), hi);
    const float node = lo + (float)c * h;
    f = ((xw == xc) ? two_sum_fraction(t, node, xl) : (xc - node)) * ih;
}

// Corner values an atom reads: v[m][4 dz + 2 dy + dx] for the atom's type map
// (m = 0), the electrostatic map (1) and the desolvation map (2). The loads
// are issued early (grid_load) and consumed later (grid_term), so that their
// latency overlaps other work.
struct GridTaps {
    float v[3][8];
    int cell[3];
};

__device__ __forceinline__ int axis_index(float t, float xl, float lo, float hi, float ih, int n) {
    const float xc = fminf(fmaxf(t + xl, lo), hi);
    return min(max((int)floorf((xc - lo) * ih), 0), n - 2);
}

// ANY_LAYOUT: the maps may be plain or corner-expanded (checked at run time);
// otherwise the corner-expanded copy is bound (the host makes sure), and the
// plain path is not compiled in (it costs registers).
template <bool ANY_LAYOUT>
__device__ __forceinline__ void grid_load(const GridParams& G, int cls, const float xl[3],
                                          const float t[3], GridTaps& tp) {
    const float ih = G.inv_spacing;
    const int cx = axis_index(t[0], xl[0], G.origin[0], G.hi[0], ih, G.nx);
    const int cy = axis_index(t[1], xl[1], G.origin[1], G.hi[1], ih, G.ny);
    const int cz = axis_index(t[2], xl[2], G.origin[2], G.hi[2], ih, G.nz);
    tp.cell[0] = cx;
    tp.cell[1] = cy;
    tp.cell[2] = cz;
    if (!ANY_LAYOUT || G.corners) {
        // corner-expanded maps: for the atom's type and cell, the 8 corners of
        // its type map, of the electrostatic and of the desolvation map are 96
        // contiguous bytes of a 128-byte block (one cache line), six 16-byte
        // loads instead of twelve rows (same values)
        const int ncx = G.nx - 1, ncy = G.ny - 1;
        const size_t ncell = (size_t)ncx * ncy * (G.nz - 1);
        const size_t cell = (size_t)((cz * ncy + cy) * ncx + cx);
        const auto base = gmem(reinterpret_cast<const f32x4*>(G.corners)) + ((size_t)cls * ncell + cell) * 8;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const f32x4 a = base[2 * m], b = base[2 * m + 1];
            tp.v[m][0] = a.x; tp.v[m][1] = a.y; tp.v[m][2] = a.z; tp.v[m][3] = a.w;
            tp.v[m][4] = b.x; tp.v[m][5] = b.y; tp.v[m][6] = b.z; tp.v[m][7] = b.w;
        }
        return;
    }
    if constexpr (!ANY_LAYOUT) return;
    const int plane = G.nx * G.ny;
    const int vol = plane * G.nz;
    const int base = (cz * G.ny + cy) * G.nx + cx;
    const auto mc = gmem(G.maps + (size_t)cls * vol + base);
    const auto me = gmem(G.maps + (size_t)(G.n_maps - 2) * vol + base);
    const auto md = gmem(G.maps + (size_t)(G.n_maps - 1) * vol + base);
    const int off[8] = {0, 1, G.nx, G.nx + 1, plane, plane + 1, plane + G.nx, plane + G.nx + 1};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        tp.v[0][i] = mc[off[i]];
        tp.v[1][i] = me[off[i]];
        tp.v[2][i] = md[off[i]];
    }
}

// Corner expansion of a grid set: thread t handles cell t % ncell for atom
// type t / ncell and writes the cell's 8 corner values (v[4 dz + 2 dy + dx])
// of that type's map, of the electrostatic map and of the desolvation map,
// as six float4 of a block of eight (the last two are zero padding, so a
// block fills one 128-byte line). Every corner index stays inside the maps
// (cells stop one node before each upper face).
__global__ __launch_bounds__(256) void expand_corners_kernel(GridParams G, float4* __restrict__ out,
                                                             long long total) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int ncx = G.nx - 1, ncy = G.ny - 1;
    const long long ncell = (long long)ncx * ncy * (G.nz - 1);
    const int type = (int)(t / ncell);
    const long long cell = t - (long long)type * ncell;
    const int cx = (int)(cell % ncx);
    const long long rest = cell / ncx;
    const int cy = (int)(rest % ncy), cz = (int)(rest / ncy);
    const size_t plane = (size_t)G.nx * G.ny;
    const size_t at = ((size_t)cz * G.ny + cy) * G.nx + cx;
    const int maps[3] = {type, G.n_maps - 2, G.n_maps - 1};
    for (int m = 0; m < 3; ++m) {
        const float* p = G.maps + (size_t)maps[m] * plane * G.nz + at;
        out[8 * t + 2 * m] = make_float4(p[0], p[1], p[G.nx], p[G.nx + 1]);
        out[8 * t + 2 * m + 1] = make_float4(p[plane], p[plane + 1], p[plane + G.nx], p[plane + G.nx + 1]);
    }
    out[8 * t + 6] = make_float4(0.f, 0.f, 0.f, 0.f);
    out[8 * t + 7] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__device__ __forceinline__ void grid_term(const GridParams& G, const GridTaps& tp, float q, float aq,
                                          const float xl[3], const float t[3],
                                          float& e, float& gx, float& gy, float& gz) {
    float fx, fy, fz, xw, yw, zw, xc, yc, zc;
    const float ih = G.inv_spacing;
    axis_cell(t[0], xl[0], G.origin[0], G.hi[0], G.spacing, ih, tp.cell[0], fx, xw, xc);
    axis_cell(t[1], xl[1], G.origin[1], G.hi[1], G.spacing, ih, tp.cell[1], fy, yw, yc);
    axis_cell(t[2], xl[2], G.origin[2], G.hi[2], G.spacing, ih, tp.cell[2], fz, zw, zc);
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = tp.v[0][i] + q * tp.v[1][i] + aq * tp.v[2][i];
    // v index = 4 dz + 2 dy + dx
    const float d00 = v[1] - v[0], d01 = v[3] - v[2], d10 = v[5] - v[4], d11 = v[7] - v[6];
    const float a00 = v[0] + fx * d00, a01 = v[2] + fx * d01;
    const float a10 = v[4] + fx * d10, a11 = v[6] + fx * d11;
    const float b0 = a00 + fy * (a01 - a00), b1 = a10 + fy * (a11 - a10);
    const float val = b0 + fz * (b1 - b0);
    const float dfz = b1 - b0;
    const float dfy = (a01 - a00) + fz * ((a11 - a10) - (a01 - a00));
    const float dx0 = d00 + fy * (d01 - d00), dx1 = d10 + fy * (d11 - d10);
    const float dfx = dx0 + fz * (dx1 - dx0);
    const float ox = xw - xc, oy = yw - yc, oz = zw - zc;
    e = val + kOut * (ox * ox + oy * oy + oz * oz);
    gx = (xw == xc ? dfx * ih : 0.f) + 2.f * kOut * ox;
    gy = (yw == yc ? dfy * ih : 0.f) + 2.f * kOut * oy;
    gz = (zw == zc ? dfz * ih : 0.f) + 2.f * kOut * oz;
}

// ---------------------------------------------------------------------------
// One pair: energy e and w = (dE/dr)/r from the separation d = x_b - x_a.
// Both dispersion-repulsion forms are A / r^12 + B / r^m, with A = eps a
// r0^12 and B = eps b r0^m taken from the pair record: 12-6
// (a, b, m) = (1, -2, 6), 12-10 hydrogen bond (5, -6, 10); r dE/dr is
// -12 A / r^12 - m B / r^m. `live` masks pairs that are not kept (e = w = 0)
// and `slope` masks the slope where r^2 is clamped (selects, so a masked
// NaN or infinity gives 0 too).
// ---------------------------------------------------------------------------

__device__ __forceinline__ void pair_term(float dx, float dy, float dz, float A, float B, bool hb,
                                          float qq, float ds, bool live, float& e, float& w) {
    const float r2raw = dx * dx + dy * dy + dz * dz;
    const bool slope = live && (r2raw >= kR2Min);
    const float r2 = fmaxf(r2raw, kR2Min);
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float ir2 = rinv * rinv;
    const float r = r2 * rinv;
    const float i4 = ir2 * ir2;
    const float i6 = i4 * ir2;
    const float i12 = i6 * i6;
    const float im = hb ? i6 * i4 : i6;
    const float t12 = A * i12;
    const float tm = B * im;
    float elj = t12 + tm;
    float dlj = -12.f * t12 + (hb ? -10.f : -6.f) * tm;                       // r dE/dr
    const bool capped = elj > kCap;
    elj = capped ? kCap : elj;
    dlj = capped ? 0.f : dlj;
    // Mehler-Solmajer dielectric eps(r) = A' + B' / D, D = 1 + K exp(-lambda B' r),
    // d eps / dr = lambda B'^2 K exp(-lambda B' r) / D^2. With M = D eps =
    // A' D + B' (> 0 for every r) one reciprocal q = 1 / (r D M) gives both
    // 1 / (r eps) = D^2 q and r eps' / eps = lambda B'^2 K exp(..) r^2 q.
    const float ex = __builtin_amdgcn_exp2f(-kDielLB * kLog2e * r);
    const float D = fmaf(kDielK, ex, 1.f);
    const float M = fmaf(kDielA, D, kDielB);
    const float q = __builtin_amdgcn_rcpf((r * D) * M);
    const float ired = (D * D) * q;
    const float eel = qq * ired;
    // r dE/dr = -E (1 + r eps' / eps)
    const float del = -eel * fmaf((r2 * ex) * q, kDielBKLB, 1.f);
    // desolvation ds exp(-r^2 / (2 sigma^2)), r dE/dr = -E r^2 / sigma^2
    const float eds = ds * __builtin_amdgcn_exp2f(-kDsInv2S2 * kLog2e * r2);
    e = live ? elj + eel + eds : 0.f;
    w = slope ? fmaf(eds, r2 * -kDsInvS2, dlj + del) * ir2 : 0.f;
}

// ---------------------------------------------------------------------------
// One listed pair (a packed record, see the blob layout) evaluated from the
// atom positions in LDS; the caller adds its force to the two slots.
// ---------------------------------------------------------------------------
struct PairForce {
    float w, dx, dy, dz, e;         // force on atom j is w * d, on atom i -w * d
    int si, sj;                     // byte offsets of the two accumulator slots
};

// Compile-time integer argument for the unrolled pipeline steps.
template <int V>
struct IntC { static constexpr int value = V; };

// Unused lanes (A = -0.0f) carry two slots no pair of their batch uses and
// get zero energy and force, so every lane updates its slots.
__device__ __forceinline__ PairForce pair_force(u32x4 pr, float4 pi, float4 pj) {
    PairForce o;
    const uint32_t rec = pr.x;
    const bool valid = pr.y != dockblob::kPadC12;
    const bool hb = (int)rec < 0;
    const float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
    const float qq = pi.w * pj.w;           // charges pre-scaled by sqrt(kElec)
    float e, w;
    pair_term(dx, dy, dz, __uint_as_float(pr.y), __uint_as_float(pr.z), hb, qq,
              __uint_as_float(pr.w), valid, e, w);
    o.e = e;
    o.w = w;
    o.dx = dx;
    o.dy = dy;
    o.dz = dz;
    o.si = rec & dockblob::kSlotMask;
    o.sj = (rec >> dockblob::kSlotShift) & dockblob::kSlotMask;
    return o;
}

// Accumulator slot at a byte offset (a multiple of 16) from `base`.
__device__ __forceinline__ float4* slot(float4* base, int byte_offset) {
    return reinterpret_cast<float4*>(
        __builtin_assume_aligned(reinterpret_cast<char*>(base) + byte_offset, 16));
}

// Adds -w d to slot si and +w d to slot sj, from their values read earlier.
// Slots are read and written whole (the fourth word passes through): 16-byte
// LDS accesses are served 16 lanes at a time, 12-byte ones take longer.
__device__ __forceinline__ void store_force(float4* base, const PairForce& f, float4 ai, float4 aj) {
    *slot(base, f.si) = make_float4(fmaf(-f.w, f.dx, ai.x), fmaf(-f.w, f.dy, ai.y), fmaf(-f.w, f.dz, ai.z), ai.w);
    *slot(base, f.sj) = make_float4(fmaf(f.w, f.dx, aj.x), fmaf(f.w, f.dy, aj.y), fmaf(f.w, f.dz, aj.z), aj.w);
}

// ---------------------------------------------------------------------------
// One evaluation of E and dE/dgenotype for the individual held by this wave.
// `gene` is gene `lane` (lanes >= G ignored); returns E (uniform) and writes
// this lane's gradient component to `grad`.
// ---------------------------------------------------------------------------
template <int SLOTS, int VAR, int WAVES = 1, bool ANY_LAYOUT = true, bool GRAD = true>
__device__ float evaluate(const GridParams& G, Smem<SLOTS, WAVES>& sm, const Lig<SLOTS>& L, float gene,
                          float& grad, float* atom_out) {
    const int lane = lane_id();
    const int N = L.N;
    const bool lead = WAVES == 1 || L.wv == 0;  // the wave that writes shared tables
    // rigid-body genes (uniform)
    const float tx = readlane(gene, 0), ty = readlane(gene, 1), tz = readlane(gene, 2);
    const float qw0 = readlane(gene, 3), qx0 = readlane(gene, 4), qy0 = readlane(gene, 5),
                qz0 = readlane(gene, 6);
    const float qinv = __builtin_amdgcn_rsqf(qw0 * qw0 + qx0 * qx0 + qy0 * qy0 + qz0 * qz0);
    const float qw = qw0 * qinv, qx = qx0 * qinv, qy = qy0 * qinv, qz = qz0 * qinv;
    float Rq[9];
    Rq[0] = 1.f - 2.f * (qy * qy + qz * qz);
    Rq[1] = 2.f * (qx * qy - qw * qz);
    Rq[2] = 2.f * (qx * qz + qw * qy);
    Rq[3] = 2.f * (qx * qy + qw * qz);
    Rq[4] = 1.f - 2.f * (qx * qx + qz * qz);
    Rq[5] = 2.f * (qy * qz - qw * qx);
    Rq[6] = 2.f * (qx * qz - qw * qy);
    Rq[7] = 2.f * (qy * qz + qw * qx);
    Rq[8] = 1.f - 2.f * (qx * qx + qy * qy);

    // torsion transforms: T_k(y) = R_k (y - p) + p, about the reference axis
    const float psi = __shfl(gene, (7 + lane) & 63);
    if (lead && lane < L.T) {
        float sn, cs;
        sincosf(psi, &sn, &cs);
        const float4 tp4 = sm.tor[lane][0], tu4 = sm.tor[lane][1];
        const float tp[3] = {tp4.x, tp4.y, tp4.z};
        const float ux = tu4.x, uy = tu4.y, uz = tu4.z;
        const float oc = 1.f - cs;
        float Rk[9];
        Rk[0] = cs + oc * ux * ux;      Rk[1] = oc * ux * uy - sn * uz; Rk[2] = oc * ux * uz + sn * uy;
        Rk[3] = oc * uy * ux + sn * uz; Rk[4] = cs + oc * uy * uy;      Rk[5] = oc * uy * uz - sn * ux;
        Rk[6] = oc * uz * ux - sn * uy; Rk[7] = oc * uz * uy + sn * ux; Rk[8] = cs + oc * uz * uz;
        float* o = sm.u.tk[lane];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            o[4 * r + 0] = Rk[3 * r + 0];
            o[4 * r + 1] = Rk[3 * r + 1];
            o[4 * r + 2] = Rk[3 * r + 2];
            o[4 * r + 3] = tp[r] - (Rk[3 * r] * tp[0] + Rk[3 * r + 1] * tp[1] + Rk[3 * r + 2] * tp[2]);
        }
    } else if (lead && lane == kMaxTors) {
        float4* o = reinterpret_cast<float4*>(sm.u.tk[kMaxTors]);
        o[0] = make_float4(1.f, 0.f, 0.f, 0.f);
        o[1] = make_float4(0.f, 1.f, 0.f, 0.f);
        o[2] = make_float4(0.f, 0.f, 1.f, 0.f);
    }
    lds_sync<WAVES>();
    // atom positions relative to the rotation centre: the torsions enclosing
    // the atom's fragment, innermost first (each about its reference axis,
    // which no inner torsion moves), then the rotation Rq. The translation t
    // is added only where world coordinates are needed (the grid term): pair
    // separations, torques and torsion axes are translation invariant and
    // keep the precision of the small local coordinates.
    const float tv[3] = {tx, ty, tz};
    const int n_duos = (L.max_depth + 1) >> 1;   // levels, two per LDS round trip
    float x[SLOTS][3];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int a = lane + kWave * (s + L.wv);
        float y0 = L.y0[s][0], y1 = L.y0[s][1], y2 = L.y0[s][2];
        // one word of torsion indices per four levels; two levels per LDS
        // round trip; levels past the atom's depth apply the identity, so
        // every lane takes the same (uniform) number of level pairs
        const uint32_t* row = sm.chain[L.frag[s]];
        for (int d = 0; d < n_duos; ++d) {
            const uint32_t w = row[d >> 1] >> (16 * (d & 1));
            float4 T[2][3];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const unsigned k = (w >> (8 * q)) & 255u;
                const float4* t = reinterpret_cast<const float4*>(__builtin_assume_aligned(
                    reinterpret_cast<const char*>(sm.u.tk) + __umul24(k, 48u), 16));
                T[q][0] = t[0]; T[q][1] = t[1]; T[q][2] = t[2];
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                // one row = three FMAs, starting from the translation column
                const float z0 = fmaf(T[q][0].x, y0, fmaf(T[q][0].y, y1, fmaf(T[q][0].z, y2, T[q][0].w)));
                const float z1 = fmaf(T[q][1].x, y0, fmaf(T[q][1].y, y1, fmaf(T[q][1].z, y2, T[q][1].w)));
                const float z2 = fmaf(T[q][2].x, y0, fmaf(T[q][2].y, y1, fmaf(T[q][2].z, y2, T[q][2].w)));
                y0 = z0; y1 = z1; y2 = z2;
            }
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) x[s][r] = Rq[3 * r] * y0 + Rq[3 * r + 1] * y1 + Rq[3 * r + 2] * y2;
        // entries past the last atom hold zeros (unused pair lanes may read them)
        sm.dyn[a] = a < N ? make_float4(x[s][0], x[s][1], x[s][2], kSqrtElec * L.chg[s][1])
                          : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    lds_sync<WAVES>();

    float g[SLOTS][3];
    float e_lane = 0.f;
    GridTaps tap[SLOTS];

    // pair terms: batches of 64 listed pairs, one per lane. Each lane adds
    // its pair's force to both atoms' accumulator slots; the host schedule
    // makes the slots of one batch distinct, so no two lanes of an
    // instruction touch one address and the order of additions is fixed.
    // (LDS float atomics would serialise in the LDS unit: they made this
    // phase several times slower.)
    if constexpr (!GRAD) {
        // energies only (a search that needs no gradient): each lane sums its
        // pairs' energies from the positions, in batch order; no
        // accumulators, no force. Software pipeline: step k reads the
        // positions of batch k + 1 from LDS before computing batch k, and
        // loads the record of batch k + 4 (records live four steps, positions
        // two; register sets indexed by k mod 4 and mod 2, steps unrolled by
        // four). Prefetch indices are clamped to the last batch.
        static_assert(WAVES == 1, "the energy-only evaluation is one wave per individual");
        const int nb = L.n_batches;
        const int pmask = L.pmask;
        auto pos_i = [&](uint32_t w) { return *slot(sm.dyn, w & pmask); };
        auto pos_j = [&](uint32_t w) { return *slot(sm.dyn, (w >> dockblob::kSlotShift) & pmask); };
        if (nb > 0) {
            const __amdgpu_buffer_rsrc_t prsrc = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<u32x4*>(L.plist), 0, nb * kWave * (int)sizeof(u32x4), kBufferWord3);
            const int lane_off = lane * (int)sizeof(u32x4);
            auto record = [&](int b) -> u32x4 {
                return __builtin_amdgcn_raw_buffer_load_b128(
                    prsrc, lane_off, uniform(min(b, nb - 1)) * kWave * (int)sizeof(u32x4), 0);
            };
            u32x4 R[4];
            float4 Pi[2], Pj[2];
#pragma unroll
            for (int q = 0; q < 4; ++q) R[q] = record(q);
            Pi[0] = pos_i(R[0].x);
            Pj[0] = pos_j(R[0].x);
            int k = 0;
            auto step = [&](auto residue, auto load) {
                constexpr int r = decltype(residue)::value;  // k mod 4
                constexpr int c = r & 1, n = (r + 1) & 1;
                const u32x4 rn = R[(r + 1) & 3];
                Pi[n] = pos_i(rn.x);
                Pj[n] = pos_j(rn.x);
                __builtin_amdgcn_sched_barrier(0);   // keep the position reads at the step's start
                e_lane += pair_force(R[r], Pi[c], Pj[c]).e;
                if constexpr (decltype(load)::value != 0) R[r] = record(k + 4);
                __builtin_amdgcn_sched_barrier(0);
                ++k;
            };
            using I0 = IntC<0>;
            using I1 = IntC<1>;
            using I2 = IntC<2>;
            using I3 = IntC<3>;
            using Load = IntC<1>;
            using NoLoad = IntC<0>;
            while (k + 4 <= nb) { step(I0(), Load()); step(I1(), Load()); step(I2(), Load()); step(I3(), Load()); }
            // the grid-map loads follow the last record load (global loads
            // complete in order)
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) grid_load<ANY_LAYOUT>(G, L.cls[s], x[s], tv, tap[s]);
            __builtin_amdgcn_sched_barrier(0);
            if (k < nb) step(I0(), NoLoad());
            if (k < nb) step(I1(), NoLoad());
            if (k < nb) step(I2(), NoLoad());
        } else {
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) grid_load<ANY_LAYOUT>(G, L.cls[s], x[s], tv, tap[s]);
        }
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) g[s][0] = g[s][1] = g[s][2] = 0.f;
    } else {
        // each wave adds into its own range of copies; with several waves per
        // individual, wave w takes the w-th of WAVES consecutive runs of
        // ceil(n_batches / WAVES) batches (the last runs may be short or empty)
        const int nslot = L.n_copies * L.stride;
        float4* const accw = sm.u.acc + (WAVES == 1 ? 0 : L.wv * nslot);
        for (int k = lane; k < nslot; k += kWave) accw[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        lds_sync<WAVES>();
        const int nb_all = L.n_batches;
        const int run = (nb_all + WAVES - 1) / WAVES;
        const int b0 = WAVES == 1 ? 0 : min(L.wv * run, nb_all);
        const int nb = WAVES == 1 ? nb_all : min(nb_all - b0, run);
        const u32x4* const plist_at = L.plist + b0 * kWave;
        const int pmask = L.pmask;
        // an atom's position sits at its slot's byte offset masked to one stride
        auto pos_i = [&](uint32_t w) { return *slot(sm.dyn, w & pmask); };
        auto pos_j = [&](uint32_t w) { return *slot(sm.dyn, (w >> dockblob::kSlotShift) & pmask); };
        // Software pipeline over batches with no branch inside. Step k
        // stores batch k (its slot values were read in step k - 1) and
        // computes batch k + 1 while reading the positions of batch k + 2
        // and loading the record of batch k + 4. A record lives four steps
        // and positions, forces and slot values two, so the steps are
        // unrolled by four with register sets indexed by the batch number
        // mod 4 and mod 2: no loaded value is copied between steps. Slot
        // updates stay in batch order (LDS executes a wave's accesses in
        // order: batch k's stores precede batch k + 1's loads). Prefetch
        // indices are clamped to the last batch, so loads need no guard.
        if (nb > 0) {
            // records through a buffer resource over this wave's batches: the
            // row offset is a scalar and the lane offset a loop-invariant
            // register, so a record load costs no vector address arithmetic
            const __amdgpu_buffer_rsrc_t prsrc = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<u32x4*>(plist_at), 0, nb * kWave * (int)sizeof(u32x4), kBufferWord3);
            const int lane_off = lane * (int)sizeof(u32x4);
            auto record = [&](int b) -> u32x4 {
                return __builtin_amdgcn_raw_buffer_load_b128(
                    prsrc, lane_off, uniform(min(b, nb - 1)) * kWave * (int)sizeof(u32x4), 0);
            };
            u32x4 R[4];
            float4 Pi[2], Pj[2], Ai[2], Aj[2];
            PairForce F[2];
#pragma unroll
            for (int q = 0; q < 4; ++q) R[q] = record(q);
            // the prologue issues its LDS reads in the loop's order (positions
            // of the next batch before the slots of this one), so that at the
            // loop head the slot reads may still be in flight
            Pi[0] = pos_i(R[0].x);
            Pj[0] = pos_j(R[0].x);
            Pi[1] = pos_i(R[1].x);
            Pj[1] = pos_j(R[1].x);
            F[0] = pair_force(R[0], Pi[0], Pj[0]);
            Ai[0] = *slot(accw, F[0].si);
            Aj[0] = *slot(accw, F[0].sj);
            int k = 0;
            auto step = [&](auto residue, auto load) {
                constexpr int r = decltype(residue)::value;  // k mod 4
                constexpr int c = r & 1, n = (r + 1) & 1;
                const u32x4 rf = R[(r + 2) & 3];
                Pi[c] = pos_i(rf.x);
                Pj[c] = pos_j(rf.x);
                if constexpr (decltype(load)::value != 0) R[r] = record(k + 4);
                __builtin_amdgcn_sched_barrier(0);   // keep the loads at the step's start
                F[n] = pair_force(R[(r + 1) & 3], Pi[n], Pj[n]);
                store_force(accw, F[c], Ai[c], Aj[c]);
                e_lane += F[c].e;
                Ai[n] = *slot(accw, F[n].si);
                Aj[n] = *slot(accw, F[n].sj);
                __builtin_amdgcn_sched_barrier(0);
                ++k;
            };
            using I0 = IntC<0>;
            using I1 = IntC<1>;
            using I2 = IntC<2>;
            using I3 = IntC<3>;
            using Load = IntC<1>;
            using NoLoad = IntC<0>;
            while (k + 4 < nb) { step(I0(), Load()); step(I1(), Load()); step(I2(), Load()); step(I3(), Load()); }
            // Every record the remaining steps need is loaded. The grid-map
            // loads go here, after the last record load: global loads
            // complete in order, so a record load issued after them would
            // wait for them. They are consumed after the pair phase.
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) grid_load<ANY_LAYOUT>(G, L.cls[s], x[s], tv, tap[s]);
            __builtin_amdgcn_sched_barrier(0);
            if (k < nb - 1) step(I0(), NoLoad());
            if (k < nb - 1) step(I1(), NoLoad());
            if (k < nb - 1) step(I2(), NoLoad());
            // k == nb - 1: the last batch is computed and its slots read
            if (k & 1) {
                store_force(accw, F[1], Ai[1], Aj[1]);
                e_lane += F[1].e;
            } else {
                store_force(accw, F[0], Ai[0], Aj[0]);
                e_lane += F[0].e;
            }
        } else {
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) grid_load<ANY_LAYOUT>(G, L.cls[s], x[s], tv, tap[s]);
        }
        lds_sync<WAVES>();
        // each atom adds its copies in copy order (range by range)
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int a = lane + kWave * (s + L.wv);
            g[s][0] = g[s][1] = g[s][2] = 0.f;
            if (a < N) {
                for (int c = 0; c < L.n_copies * WAVES; ++c) {
                    const float4 v = sm.u.acc[c * L.stride + a];
                    g[s][0] += v.x;
                    g[s][1] += v.y;
                    g[s][2] += v.z;
                }
            }
        }
    }
    // grid term, from the corner values loaded before the pair phase
    float e_atom[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int a = lane + kWave * (s + L.wv);
        float e, gx, gy, gz;
        grid_term(G, tap[s], L.chg[s][1], L.chg[s][2], x[s], tv, e, gx, gy, gz);
        const bool ok = a < N;
        e_atom[s] = ok ? e : 0.f;
        g[s][0] += ok ? gx : 0.f;
        g[s][1] += ok ? gy : 0.f;
        g[s][2] += ok ? gz : 0.f;
        e_lane += e_atom[s];
    }
#pragma unroll
    for (int s = 0; s < SLOTS; ++s)
        if (lane + kWave * (s + L.wv) >= N) { g[s][0] = g[s][1] = g[s][2] = 0.f; }

    if constexpr (!GRAD) {
        // the block sum of E alone, in the chosen variant
        grad = 0.f;
        lds_sync<WAVES>();   // the next evaluation rewrites the position table
        return sum4<VAR>(make_float4(e_lane, 0.f, 0.f, 0.f)).x;
    }

    // block sum of {E, gx, gy, gz}: the paper's reduction, in the chosen variant
    float4 eg = make_float4(e_lane, 0.f, 0.f, 0.f);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) { eg.y += g[s][0]; eg.z += g[s][1]; eg.w += g[s][2]; }
    float4 EG = sum4<VAR>(eg);

    // torsion torques: prefix sums of (g, x cross g) in depth-first order;
    // the last lane's x cross g sums give the torque about t (FP32 always)
    float P[SLOTS][6];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        P[s][0] = g[s][0]; P[s][1] = g[s][1]; P[s][2] = g[s][2];
        P[s][3] = x[s][1] * g[s][2] - x[s][2] * g[s][1];
        P[s][4] = x[s][2] * g[s][0] - x[s][0] * g[s][2];
        P[s][5] = x[s][0] * g[s][1] - x[s][1] * g[s][0];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        P[0][c] = wave_scan(P[0][c]);
        if constexpr (SLOTS == 2) P[1][c] = wave_scan(P[1][c]) + readlane(P[0][c], 63);
    }
    float4 TQ = make_float4(readlane(P[SLOTS - 1][3], 63), readlane(P[SLOTS - 1][4], 63),
                            readlane(P[SLOTS - 1][5], 63), 0.f);
    if constexpr (WAVES > 1) {
        // the waves' partials and prefix sums meet in LDS; every wave then
        // holds the same totals (added in wave order) and steps identically
        const int a = lane + kWave * L.wv;
#pragma unroll
        for (int c = 0; c < 6; ++c) sm.pre[c][a] = P[0][c];
        if (lane == 0) sm.xchg[L.wv][0] = EG;
        lds_sync<WAVES>();
        EG = sm.xchg[0][0];
        TQ = make_float4(sm.pre[3][kWave - 1], sm.pre[4][kWave - 1], sm.pre[5][kWave - 1], 0.f);
#pragma unroll
        for (int w = 1; w < WAVES; ++w) {
            const float4 ew = sm.xchg[w][0];
            EG = make_float4(EG.x + ew.x, EG.y + ew.y, EG.z + ew.z, EG.w + ew.w);
            TQ = make_float4(TQ.x + sm.pre[3][(w + 1) * kWave - 1], TQ.y + sm.pre[4][(w + 1) * kWave - 1],
                             TQ.z + sm.pre[5][(w + 1) * kWave - 1], 0.f);
        }
    }
    float gpsi = 0.f;
    {
        // torsion `lane`: bond atoms a, b and its moving range [first, end)
        // in depth-first positions; lanes without a torsion read a harmless
        // default (a = b = 0, empty range at 1)
        const int pk = lane < L.T ? __float_as_int(sm.tor[lane & (kMaxTors - 1)][0].w) : (1 << 16) | (1 << 24);
        const int t_apos = pk & 255, t_bpos = (pk >> 8) & 255;
        const int hi = ((pk >> 24) & 255) - 1, lo = ((pk >> 16) & 255) - 1;
        float S[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            if constexpr (WAVES > 1) {
                // global prefix: a wave's local prefix plus the totals of the
                // waves before it (added in wave order)
                const float bh = sm.pre[c][hi], bl = sm.pre[c][lo];
                float ph = bh, pl = bl, off = 0.f;
#pragma unroll
                for (int w = 1; w < WAVES; ++w) {
                    off = w == 1 ? sm.pre[c][kWave - 1] : off + sm.pre[c][w * kWave - 1];
                    ph = hi >= w * kWave ? bh + off : ph;
                    pl = lo >= w * kWave ? bl + off : pl;
                }
                S[c] = ph - pl;
            } else {
                float ph = __shfl(P[0][c], hi & 63);
                float pl = __shfl(P[0][c], lo & 63);
                if constexpr (SLOTS == 2) {
                    const float ph1 = __shfl(P[1][c], hi & 63);
                    const float pl1 = __shfl(P[1][c], lo & 63);
                    ph = hi >= kWave ? ph1 : ph;
                    pl = lo >= kWave ? pl1 : pl;
                }
                S[c] = ph - pl;
            }
        }
        const float4 xa = sm.dyn[t_apos];
        const float4 xb = sm.dyn[t_bpos];
        float ux = xb.x - xa.x, uy = xb.y - xa.y, uz = xb.z - xa.z;
        const float il = __builtin_amdgcn_rsqf(ux * ux + uy * uy + uz * uz);
        ux *= il; uy *= il; uz *= il;
        // S_xg - x_a cross S_g
        const float mx = S[3] - (xa.y * S[2] - xa.z * S[1]);
        const float my = S[4] - (xa.z * S[0] - xa.x * S[2]);
        const float mz = S[5] - (xa.x * S[1] - xa.y * S[0]);
        gpsi = (lane < L.T) ? ux * mx + uy * my + uz * mz : 0.f;
    }
    // gradient with respect to the genotype
    {
        // (2/|q|) (0, tau) (x) q_hat
        const float k2 = 2.0f * qinv;
        const float gw = -(TQ.x * qx + TQ.y * qy + TQ.z * qz);
        const float gqx = qw * TQ.x + (TQ.y * qz - TQ.z * qy);
        const float gqy = qw * TQ.y + (TQ.z * qx - TQ.x * qz);
        const float gqz = qw * TQ.z + (TQ.x * qy - TQ.y * qx);
        const float gt = __shfl(gpsi, (lane - 7) & 63);
        float gr = gt;
        gr = lane == 0 ? EG.y : gr;
        gr = lane == 1 ? EG.z : gr;
        gr = lane == 2 ? EG.w : gr;
        gr = lane == 3 ? k2 * gw : gr;
        gr = lane == 4 ? k2 * gqx : gr;
        gr = lane == 5 ? k2 * gqy : gr;
        gr = lane == 6 ? k2 * gqz : gr;
        grad = gr;
    }
    if (atom_out) {
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int a = lane + kWave * (s + L.wv);
            if (a < N) {
                float4* o = reinterpret_cast<float4*>(atom_out) + 2 * L.orig[s];
                // position relative to t, as held (t + it is the world position)
                o[0] = make_float4(x[s][0], x[s][1], x[s][2], e_atom[s]);
                o[1] = make_float4(g[s][0], g[s][1], g[s][2], 0.f);
            }
        }
    }
    return EG.x;
}

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------

// Persistent scoring kernel: each wave loads the ligand once (LDS tables and
// per-lane registers) and evaluates genotypes ind = blockIdx.x,
// blockIdx.x + gridDim.x, ... (independent evaluations, so a static stride
// gives the same results as any other assignment). ANY_LAYOUT: the maps may
// be plain or corner-expanded; otherwise the corner-expanded copy is bound.
template <int SLOTS, int VAR, bool ANY_LAYOUT>
__global__ __launch_bounds__(64, (SLOTS == 1 ? 3 : 2)) void score_kernel(GridParams G, const uint8_t* __restrict__ blob,
                                                   int n, const float* __restrict__ gen,
                                                   float* __restrict__ energy,
                                                   float* __restrict__ grad,
                                                   float* __restrict__ atom_out) {
    __shared__ Smem<SLOTS> sm;
    Lig<SLOTS> L;
    load_ligand<SLOTS>(blob, sm, L);
    const int lane = lane_id();
    const int G_ = L.G;
    for (int ind = blockIdx.x; ind < n; ind += gridDim.x) {
        const float gene = lane < G_ ? gen[(size_t)ind * G_ + lane] : 0.f;
        float gr;
        float* ao = atom_out ? atom_out + (size_t)ind * L.N * 8 : nullptr;
        const float E = evaluate<SLOTS, VAR, 1, ANY_LAYOUT>(G, sm, L, gene, gr, ao);
        if (lane == 0) energy[ind] = E;
        if (grad && lane < G_) grad[(size_t)ind * G_ + lane] = gr;
    }
}

// Solis-Wets random search (Sec. 2.1: the LGA's second local search; the
// steps are those of Solis and Wets as AutoDock uses them): per iteration the
// trial x + bias + dev, else x - bias - dev, accepted when its energy is lower;
// bias and the step scale rho follow the outcome. One wave per individual,
// gene `lane`; energies only (the gradient evaluate() also makes is unused).
// State updates are float32 in a fixed order with no fused operations
// (contraction is off in this kernel; evaluate() keeps its own FMAs).
template <int SLOTS, int VAR>
__global__ __launch_bounds__(64, (SLOTS == 1 ? 3 : 2)) void sw_kernel(GridParams G, const uint8_t* __restrict__ blob,
                                                docklaunch::SwParams p) {
    // no product below may be fused into an add (FMA): the state must round
    // after every operation
#pragma clang fp contract(off)
    __shared__ Smem<SLOTS> sm;
    Lig<SLOTS> L;
    load_ligand<SLOTS>(blob, sm, L);
    const int lane = lane_id();
    const int ind = blockIdx.x;
    if (ind >= p.n) return;
    const int Gn = L.G;
    const bool on = lane < Gn;
    const size_t row = (size_t)ind * Gn + lane;
    float x = on ? p.genotype[row] : 0.f;
    float b = on ? p.bias[row] : 0.f;
    const float sc = on ? p.scale[lane] : 0.f;
    float E = p.energy[ind];
    float rho = p.rho[ind];
    int succ = p.counts[2 * ind], fail = p.counts[2 * ind + 1];
    for (int it = 0; it < p.iterations; ++it) {
        const float z = on ? p.normals[((size_t)it * p.n + ind) * Gn + lane] : 0.f;
        const float dev = rho * (sc * z);
        float e_try0 = __builtin_nanf(""), e_try1 = __builtin_nanf("");
        int accepted = -1;
        for (int t = 0; t < 2; ++t) {      // uniform: E and the trial energies are wave-uniform
            const float c = t == 0 ? (x + b) + dev : (x - b) - dev;
            float gr;
            const float Et = evaluate<SLOTS, VAR, 1, true, false>(G, sm, L, c, gr, nullptr);
            if (t == 0) e_try0 = Et; else e_try1 = Et;
            if (Et < E) {
                x = c;
                E = Et;
                accepted = t;
                break;
            }
        }
        if (accepted == 0) {
            b = 0.2f * b + 0.4f * dev;
            ++succ;
            fail = 0;
        } else if (accepted == 1) {
            b = b - 0.4f * dev;
            ++succ;
            fail = 0;
        } else {
            b = 0.5f * b;
            ++fail;
            succ = 0;
        }
        if (succ >= p.n_success) {
            rho = 2.f * rho;
            succ = 0;
        } else if (fail >= p.n_failure) {
            rho = 0.5f * rho;
            fail = 0;
        }
        if (p.log && lane == 0) {
            p.log[((size_t)ind * p.iterations + it) * 2] = e_try0;
            p.log[((size_t)ind * p.iterations + it) * 2 + 1] = e_try1;
        }
    }
    if (on) {
        p.genotype[row] = x;
        p.bias[row] = b;
    }
    if (lane == 0) {
        p.energy[ind] = E;
        p.rho[ind] = rho;
        p.counts[2 * ind] = succ;
        p.counts[2 * ind + 1] = fail;
    }
}

template <int SLOTS, int VAR, int WAVES = 1, bool ANY_LAYOUT = true>
__device__ void local_search_one(const DevItem& it, int ind, Smem<SLOTS, WAVES>& sm, const Lig<SLOTS>& L,
                                 int iterations, float rho, float eps, bool final_eval) {
    // with several waves per individual every wave holds the genotype and
    // takes the same steps on the same totals; the first wave writes the
    // results
    const int lane = lane_id();
    const bool writer = WAVES == 1 || L.wv == 0;
    const int G = L.G;
    const bool act = lane < G;
    const size_t o = (size_t)ind * G + lane;
    float x = act ? it.genotype[o] : 0.f;
    float ag = act ? it.acc_g2[o] : 0.f;
    float ad = act ? it.acc_dx2[o] : 0.f;
    float bx = act ? it.best_genotype[o] : 0.f;
    float bestE = it.best_energy[ind];
    float lastE = it.energy[ind];
    float lastG = 0.f;
    for (int iter = 0; iter < iterations; ++iter) {
        float gr;
        const float E = evaluate<SLOTS, VAR, WAVES, ANY_LAYOUT>(it.grid, sm, L, x, gr, nullptr);
        lastE = E;
        lastG = gr;
        if (E < bestE) { bestE = E; bx = x; }
        gr = act ? gr : 0.f;
        ag = rho * ag + (1.f - rho) * gr * gr;
        const float dx = -(__builtin_amdgcn_sqrtf(ad + eps) * __builtin_amdgcn_rsqf(ag + eps)) * gr;
        ad = rho * ad + (1.f - rho) * dx * dx;
        float xn = x + dx;
        const bool isq = lane >= 3 && lane < 7;
        const float q2 = isq ? xn * xn : 0.f;
        const float nq2 = (readlane(q2, 3) + readlane(q2, 4)) + (readlane(q2, 5) + readlane(q2, 6));
        if (isq) xn = (nq2 >= 1e-12f) ? xn * __builtin_amdgcn_rsqf(nq2) : x;
        x = act ? xn : 0.f;
    }
    if (final_eval) {
        float gr;
        const float E = evaluate<SLOTS, VAR, WAVES, ANY_LAYOUT>(it.grid, sm, L, x, gr, nullptr);
        lastE = E;
        lastG = gr;
        if (E < bestE) { bestE = E; bx = x; }
    }
    if (!writer) return;
    if (act && it.grad && (iterations > 0 || final_eval)) it.grad[o] = lastG;
    if (act) {
        it.genotype[o] = x;
        it.acc_g2[o] = ag;
        it.acc_dx2[o] = ad;
        it.best_genotype[o] = bx;
    }
    if (lane == 0) {
        it.best_energy[ind] = bestE;
        it.energy[ind] = lastE;
        it.iters_done[ind] += iterations;
    }
}

template <int SLOTS, int WAVES>
__device__ void ls_dispatch(int var_uniform, const DevItem& it, int ind, Smem<SLOTS, WAVES>& sm,
                            const Lig<SLOTS>& L, const LsParams& p) {
    const int var = var_uniform >= 0 ? var_uniform : it.variant;
    const bool fin = it.final_eval != 0;
    switch (var) {
        case DOCK_REDUCE_MFMA_F32:
            local_search_one<SLOTS, DOCK_REDUCE_MFMA_F32, WAVES>(it, ind, sm, L, it.iterations, p.rho, p.eps, fin); break;
        case DOCK_REDUCE_MFMA_BF16:
            local_search_one<SLOTS, DOCK_REDUCE_MFMA_BF16, WAVES>(it, ind, sm, L, it.iterations, p.rho, p.eps, fin); break;
        case DOCK_REDUCE_MFMA_F16:
            local_search_one<SLOTS, DOCK_REDUCE_MFMA_F16, WAVES>(it, ind, sm, L, it.iterations, p.rho, p.eps, fin); break;
        case DOCK_REDUCE_MFMA_BF16X3:
            local_search_one<SLOTS, DOCK_REDUCE_MFMA_BF16X3, WAVES>(it, ind, sm, L, it.iterations, p.rho, p.eps, fin); break;
        default:
            local_search_one<SLOTS, DOCK_REDUCE_SHUFFLE, WAVES>(it, ind, sm, L, it.iterations, p.rho, p.eps, fin); break;
    }
}

template <int SLOTS, int VAR, int WAVES = 1>
__device__ void ls_run(const DevItem& it, int ind, Smem<SLOTS, WAVES>& sm, const Lig<SLOTS>& L,
                       const LsParams& p) {
    // a kernel specialised for one variant runs only items whose grids have
    // the corner-expanded copy bound; the dispatching kernel takes any
    if constexpr (VAR >= 0)
        local_search_one<SLOTS, VAR, WAVES, false>(it, ind, sm, L, it.iterations, p.rho, p.eps, it.final_eval != 0);
    else
        ls_dispatch<SLOTS, WAVES>(-1, it, ind, sm, L, p);
}

// The item of work unit u: the last item with unit_begin <= u (items are
// in unit order).
__device__ __forceinline__ int item_of_unit(const LsParams& p, int u) {
    int lo = 0, hi = p.n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (uniform(gmem(&p.items[mid].unit_begin)[0]) <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The item record, read once per work unit, with every word made
// wave-uniform (scalar registers).
__device__ __forceinline__ DevItem load_item(const DevItem* items, int k) {
    static_assert(sizeof(DevItem) % 4 == 0, "item record is made of 32-bit words");
    constexpr int kWords = sizeof(DevItem) / 4;
    const auto src = gmem(reinterpret_cast<const uint32_t*>(items + k));
    DevItem out;
    uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
    for (int w = 0; w < kWords; ++w) dst[w] = __builtin_amdgcn_readfirstlane(src[w]);
    return out;
}

// Persistent local-search kernel. Work units are individuals, numbered item by
// item in the order the host gives (longest items first); each wave takes the
// next unit from a global counter until none is left, reloading the ligand
// only when the item changes. Every wave exits once the counter passes the
// last unit.
template <int MODE, int VAR>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MODE == docklaunch::kSlots1 ? 3 : 2, MODE == docklaunch::kSlots1 ? 3 : 2))) void ls_kernel(LsParams p) {
    // LDS sized for the layouts the launch can meet
    constexpr size_t kBytes = MODE == docklaunch::kSlots1 ? sizeof(Smem<1>) : sizeof(Smem<2>);
    __shared__ __align__(16) unsigned char smem[kBytes];
    int cur_item = -1;
    while (true) {
        int u = 0;
        if (lane_id() == 0) u = atomicAdd(p.counter, 1);
        u = uniform(u);
        if (u >= p.total_units) break;
        const int lo = item_of_unit(p, u);
        const DevItem it = load_item(p.items, lo);
        const int ind = u - it.unit_begin;
        // the ligand's LDS tables are refilled only when the item changes;
        // its per-lane registers are rebuilt for every individual, so that no
        // ligand state stays live across units (the two atom-slot layouts of
        // a mixed launch would otherwise both hold registers)
        const bool reload = lo != cur_item;
        cur_item = lo;
        const bool one = MODE == docklaunch::kSlots1 || (MODE == docklaunch::kSlotsAny && it.slots == 1);
        if (one) {
            Smem<1>& sm = *reinterpret_cast<Smem<1>*>(smem);
            Lig<1> L;
            load_ligand<1>(it.blob, sm, L, reload);
            ls_run<1, VAR>(it, ind, sm, L, p);
        } else if constexpr (MODE != docklaunch::kSlots1) {
            Smem<2>& sm = *reinterpret_cast<Smem<2>*>(smem);
            Lig<2> L;
            load_ligand<2>(it.blob, sm, L, reload);
            ls_run<2, VAR>(it, ind, sm, L, p);
        }
    }
}

// Persistent local-search kernel with WAVES (2 or 4) waves per individual:
// one individual per block of 64 WAVES threads, wave w owning atom positions
// 64 w .. 64 w + 63 and the w-th run of the pair batches. The first thread
// takes the next unit and hands it to every wave through LDS; every wave
// exits once the counter passes the last unit.
template <int VAR, int WAVES>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(3, 3))) void ls_kernel_mw(LsParams p) {
    __shared__ Smem<1, WAVES> sm;
    int cur_item = -1;
    while (true) {
        __syncthreads();                       // the previous unit is read by every wave
        if (threadIdx.x == 0) sm.unit = atomicAdd(p.counter, 1);
        __syncthreads();
        const int u = uniform(sm.unit);
        if (u >= p.total_units) break;
        const int lo = item_of_unit(p, u);
        const DevItem it = load_item(p.items, lo);
        const int ind = u - it.unit_begin;
        const bool reload = lo != cur_item;
        cur_item = lo;
        Lig<1> L;
        load_ligand<1, WAVES>(it.blob, sm, L, reload);
        ls_run<1, VAR, WAVES>(it, ind, sm, L, p);
    }
}

// ---------------------------------------------------------------------------
// Two individuals per wave, for ligands of at most 32 atoms and 25 torsions
// (G = 7 + T <= 32 genes): each 32-lane half of the wave holds one
// individual, lane j of half h holding atom j and gene j of individual h.
// The per-atom stages then fill twice as many lanes as with one individual
// per wave, and the per-evaluation tail (block sum, prefix scans, gradient
// assembly, update) serves two individuals. The pair phase walks the same
// 64-record batches in two steps of 32 records, each half adding forces to
// its own accumulator slots (the slots of a batch are distinct, so those of
// a half-batch are too). The block sum is the wavefront shuffle over each
// half; the halves never exchange values, so an individual's result does
// not depend on the other half.
// ---------------------------------------------------------------------------
constexpr int kHalf = 32;

// LDS of a two-individual wave. Twelve such blocks (three waves per SIMD) must
// fit in the CU's 160 KB after each block's LDS is rounded up to the
// allocation granularity: 12,800 bytes per block fit, while the 13,344 bytes
// of accumulators sized for 320 slots per half left room for eleven blocks
// per CU. A ligand of <= 32 atoms needs at most 288 slots.
struct __align__(16) Smem2 {
    float4 dyn[2][kHalf];               // per half: positions relative to t, sqrt(kElec) q
    union {
        float tk[2][kMaxTors + 1][12];  // per half: torsion transforms, identity at kMaxTors
        float4 acc[2][dockblob::kMaxSlotsTiny];   // per half: pair-force accumulators
    } u;
    float4 tor[kMaxTors][2];
    uint32_t chain[kMaxFrag][kChain / 4];
};
static_assert(sizeof(Smem2) <= 12800, "twelve two-individual blocks per CU");

__device__ __forceinline__ float hsel(float a, float b) { return lane_id() < kHalf ? a : b; }

// Lane c of this lane's half.
__device__ __forceinline__ float half_lane(float v, int c) { return hsel(readlane(v, c), readlane(v, kHalf + c)); }

// Sum over this lane's half, every lane of the half receives it: row sums by
// a DPP butterfly, then row 0 into row 1 and row 2 into row 3.
__device__ __forceinline__ float half_sum(float v) {
    v += dpp<0xB1>(v);         // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);         // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);        // row_half_mirror
    v += dpp<0x140>(v);        // row_mirror
    v += dpp<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    return hsel(readlane(v, kHalf - 1), readlane(v, 2 * kHalf - 1));
}

// Inclusive prefix sum within each half.
__device__ __forceinline__ float half_scan(float v) {
    v += dpp<0x111>(v);          // row_shr:1
    v += dpp<0x112>(v);          // row_shr:2
    v += dpp<0x114>(v);          // row_shr:4
    v += dpp<0x118>(v);          // row_shr:8
    v += dpp<0x142, 0xa>(v);     // row_bcast:15 into rows 1 and 3
    return v;
}

// The ligand as a two-individual wave holds it: lane j of either half the
// atom j (per-lane registers), the shared torsion and fragment tables in LDS.
__device__ void load_ligand2(const uint8_t* __restrict__ blob, Smem2& sm, Lig<1>& L, bool fill_lds = true) {
    if (fill_lds) wave_sync();  // previous users of the LDS tables are done
    const Header* h = reinterpret_cast<const Header*>(blob);
    const int lane = lane_id();
    L.wv = 0;
    L.N = uniform(h->n_atoms);
    L.T = uniform(h->n_torsions);
    L.NF = uniform(h->n_frag);
    L.G = uniform(h->n_genes);
    L.n_batches = uniform(h->n_batches);
    L.n_copies = uniform(h->n_copies);
    L.max_depth = uniform(h->max_depth);
    L.stride = uniform(h->slot_stride);
    L.pmask = L.stride * 16 - 1;
    L.plist = uniform_ptr(reinterpret_cast<const u32x4*>(blob + h->off_plist));
    const float4* ref = reinterpret_cast<const float4*>(blob + h->off_ref);
    const float4* chg = reinterpret_cast<const float4*>(blob + h->off_chg);
    const int4* iv = reinterpret_cast<const int4*>(blob + h->off_int);
    const int a = lane & (kHalf - 1);
    const bool ok = a < L.N;
    const int ai = ok ? a : 0;
    const float4 r = ref[ai], c = chg[ai];
    const int4 ii = iv[ai];
    L.y0[0][0] = r.x; L.y0[0][1] = r.y; L.y0[0][2] = r.z;
    L.chg[0][0] = ok ? c.x : 0.f; L.chg[0][1] = ok ? c.y : 0.f; L.chg[0][2] = ok ? c.z : 0.f;
    L.cls[0] = ii.x;
    L.frag[0] = ii.y;
    L.orig[0] = ii.z;
    const Torsion* tr = reinterpret_cast<const Torsion*>(blob + h->off_tors);
    if (fill_lds && lane < L.T) {
        const Torsion t = tr[lane];
        const int pk = t.a_pos | (t.b_pos << 8) | (t.first << 16) | (t.end << 24);
        sm.tor[lane][0] = make_float4(t.p[0], t.p[1], t.p[2], __int_as_float(pk));
        sm.tor[lane][1] = make_float4(t.u[0], t.u[1], t.u[2], 0.f);
    }
    const uint32_t* ch = reinterpret_cast<const uint32_t*>(blob + h->off_chain);
    const int n_chain_words = L.NF * (kChain / 4);
    uint32_t* dst = &sm.chain[0][0];
    if (fill_lds)
        for (int i = lane; i < n_chain_words; i += kWave) dst[i] = ch[i];
    wave_sync();
}

// One evaluation of E and dE/dgenotype for the two individuals of the wave.
// `gene` is gene j of this lane's individual (j = lane % 32; j >= G
// ignored); returns this half's E and writes this lane's gradient component
// to `grad`. atom_out: this half's per-atom output (or nullptr).
template <bool ANY_LAYOUT, bool GRAD = true>
__device__ float evaluate2(const GridParams& G, Smem2& sm, const Lig<1>& L, float gene, float& grad,
                           float* atom_out) {
    const int lane = lane_id();
    const int j = lane & (kHalf - 1);
    const int h = lane >> 5;
    const int hb = h * kHalf;
    const int N = L.N;
    const float tx = half_lane(gene, 0), ty = half_lane(gene, 1), tz = half_lane(gene, 2);
    const float qw0 = half_lane(gene, 3), qx0 = half_lane(gene, 4), qy0 = half_lane(gene, 5),
                qz0 = half_lane(gene, 6);
    const float qinv = __builtin_amdgcn_rsqf(qw0 * qw0 + qx0 * qx0 + qy0 * qy0 + qz0 * qz0);
    const float qw = qw0 * qinv, qx = qx0 * qinv, qy = qy0 * qinv, qz = qz0 * qinv;
    float Rq[9];
    Rq[0] = 1.f - 2.f * (qy * qy + qz * qz);
    Rq[1] = 2.f * (qx * qy - qw * qz);
    Rq[2] = 2.f * (qx * qz + qw * qy);
    Rq[3] = 2.f * (qx * qy + qw * qz);
    Rq[4] = 1.f - 2.f * (qx * qx + qz * qz);
    Rq[5] = 2.f * (qy * qz - qw * qx);
    Rq[6] = 2.f * (qx * qz - qw * qy);
    Rq[7] = 2.f * (qy * qz + qw * qx);
    Rq[8] = 1.f - 2.f * (qx * qx + qy * qy);

    // torsion transforms of this half's individual (T <= 25, so lane 31 of
    // each half is free to write the identity)
    const float psi = __shfl(gene, hb + ((7 + j) & (kHalf - 1)));
    if (j < L.T) {
        float sn, cs;
        sincosf(psi, &sn, &cs);
        const float4 tp4 = sm.tor[j][0], tu4 = sm.tor[j][1];
        const float tp[3] = {tp4.x, tp4.y, tp4.z};
        const float ux = tu4.x, uy = tu4.y, uz = tu4.z;
        const float oc = 1.f - cs;
        float Rk[9];
        Rk[0] = cs + oc * ux * ux;      Rk[1] = oc * ux * uy - sn * uz; Rk[2] = oc * ux * uz + sn * uy;
        Rk[3] = oc * uy * ux + sn * uz; Rk[4] = cs + oc * uy * uy;      Rk[5] = oc * uy * uz - sn * ux;
        Rk[6] = oc * uz * ux - sn * uy; Rk[7] = oc * uz * uy + sn * ux; Rk[8] = cs + oc * uz * uz;
        float* o = sm.u.tk[h][j];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            o[4 * r + 0] = Rk[3 * r + 0];
            o[4 * r + 1] = Rk[3 * r + 1];
            o[4 * r + 2] = Rk[3 * r + 2];
            o[4 * r + 3] = tp[r] - (Rk[3 * r] * tp[0] + Rk[3 * r + 1] * tp[1] + Rk[3 * r + 2] * tp[2]);
        }
    } else if (j == kHalf - 1) {
        float4* o = reinterpret_cast<float4*>(sm.u.tk[h][kMaxTors]);
        o[0] = make_float4(1.f, 0.f, 0.f, 0.f);
        o[1] = make_float4(0.f, 1.f, 0.f, 0.f);
        o[2] = make_float4(0.f, 0.f, 1.f, 0.f);
    }
    wave_sync();
    // atom positions relative to the rotation centre, as in `evaluate`
    const float tv[3] = {tx, ty, tz};
    const int n_duos = (L.max_depth + 1) >> 1;
    float x[3];
    {
        float y0 = L.y0[0][0], y1 = L.y0[0][1], y2 = L.y0[0][2];
        const uint32_t* row = sm.chain[L.frag[0]];
        const char* tkh = reinterpret_cast<const char*>(sm.u.tk[h]);
        for (int d = 0; d < n_duos; ++d) {
            const uint32_t w = row[d >> 1] >> (16 * (d & 1));
            float4 T[2][3];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const unsigned k = (w >> (8 * q)) & 255u;
                const float4* t = reinterpret_cast<const float4*>(
                    __builtin_assume_aligned(tkh + __umul24(k, 48u), 16));
                T[q][0] = t[0]; T[q][1] = t[1]; T[q][2] = t[2];
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const float z0 = fmaf(T[q][0].x, y0, fmaf(T[q][0].y, y1, fmaf(T[q][0].z, y2, T[q][0].w)));
                const float z1 = fmaf(T[q][1].x, y0, fmaf(T[q][1].y, y1, fmaf(T[q][1].z, y2, T[q][1].w)));
                const float z2 = fmaf(T[q][2].x, y0, fmaf(T[q][2].y, y1, fmaf(T[q][2].z, y2, T[q][2].w)));
                y0 = z0; y1 = z1; y2 = z2;
            }
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) x[r] = Rq[3 * r] * y0 + Rq[3 * r + 1] * y1 + Rq[3 * r + 2] * y2;
        // entries past the last atom hold zeros (unused pair lanes may read them)
        sm.dyn[h][j] = j < N ? make_float4(x[0], x[1], x[2], kSqrtElec * L.chg[0][1])
                             : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    wave_sync();

    float g[3] = {0.f, 0.f, 0.f};
    float e_lane = 0.f;
    GridTaps tap;
    float4* const dynh = sm.dyn[h];
    float4* const acch = sm.u.acc[h];
    const int pmask = L.pmask;
    auto pos_i = [&](uint32_t w) { return *slot(dynh, w & pmask); };
    auto pos_j = [&](uint32_t w) { return *slot(dynh, (w >> dockblob::kSlotShift) & pmask); };
    if constexpr (GRAD) {
        const int nslot = L.n_copies * L.stride;
        for (int k = j; k < nslot; k += kHalf) acch[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        wave_sync();
    }
    // pair terms: step s takes records 32 (s % 2) .. 32 (s % 2) + 31 of
    // batch s / 2, record j for lane j of either half. Software pipeline:
    // step s reads the positions of step s + 1 before computing its own pair
    // and loads the record of step s + 4 (register sets indexed by s mod 4
    // and mod 2, steps unrolled by four, no loaded value copied between
    // steps); prefetch indices are clamped to the last step.
    const int ns = 2 * L.n_batches;
    if (ns > 0) {
        const __amdgpu_buffer_rsrc_t prsrc = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<u32x4*>(L.plist), 0, ns * kHalf * (int)sizeof(u32x4), kBufferWord3);
        const int lane_off = j * (int)sizeof(u32x4);
        auto record = [&](int s) -> u32x4 {
            return __builtin_amdgcn_raw_buffer_load_b128(
                prsrc, lane_off, uniform(min(s, ns - 1)) * kHalf * (int)sizeof(u32x4), 0);
        };
        u32x4 R[4];
        float4 Pi[2], Pj[2];
#pragma unroll
        for (int q = 0; q < 4; ++q) R[q] = record(q);
        Pi[0] = pos_i(R[0].x);
        Pj[0] = pos_j(R[0].x);
        int s = 0;
        auto step = [&](auto residue, auto load) {
            constexpr int r = decltype(residue)::value;  // s mod 4
            constexpr int c = r & 1, n = (r + 1) & 1;
            const u32x4 rn = R[(r + 1) & 3];
            Pi[n] = pos_i(rn.x);
            Pj[n] = pos_j(rn.x);
            __builtin_amdgcn_sched_barrier(0);
            const PairForce F = pair_force(R[r], Pi[c], Pj[c]);
            if constexpr (GRAD) {
                const float4 ai = *slot(acch, F.si);
                const float4 aj = *slot(acch, F.sj);
                store_force(acch, F, ai, aj);
            }
            e_lane += F.e;
            if constexpr (decltype(load)::value != 0) R[r] = record(s + 4);
            __builtin_amdgcn_sched_barrier(0);
            ++s;
        };
        using I0 = IntC<0>;
        using I1 = IntC<1>;
        using I2 = IntC<2>;
        using I3 = IntC<3>;
        using Load = IntC<1>;
        using NoLoad = IntC<0>;
        while (s + 4 <= ns) { step(I0(), Load()); step(I1(), Load()); step(I2(), Load()); step(I3(), Load()); }
        __builtin_amdgcn_sched_barrier(0);
        grid_load<ANY_LAYOUT>(G, L.cls[0], x, tv, tap);
        __builtin_amdgcn_sched_barrier(0);
        if (s < ns) step(I0(), NoLoad());
        if (s < ns) step(I1(), NoLoad());
        if (s < ns) step(I2(), NoLoad());
    } else {
        grid_load<ANY_LAYOUT>(G, L.cls[0], x, tv, tap);
    }
    if constexpr (GRAD) {
        wave_sync();
        // each atom adds its copies in copy order
        if (j < N)
            for (int c = 0; c < L.n_copies; ++c) {
                const float4 v = acch[c * L.stride + j];
                g[0] += v.x;
                g[1] += v.y;
                g[2] += v.z;
            }
    }
    // grid term
    float e_atom;
    {
        float e, gx, gy, gz;
        grid_term(G, tap, L.chg[0][1], L.chg[0][2], x, tv, e, gx, gy, gz);
        const bool ok = j < N;
        e_atom = ok ? e : 0.f;
        g[0] = ok ? g[0] + gx : 0.f;
        g[1] = ok ? g[1] + gy : 0.f;
        g[2] = ok ? g[2] + gz : 0.f;
        e_lane += e_atom;
    }
    if constexpr (!GRAD) {
        grad = 0.f;
        wave_sync();   // the next evaluation rewrites the position table
        return half_sum(e_lane);
    }
    // block sum of {E, gx, gy, gz} over each half (wavefront shuffle)
    const float4 EG = make_float4(half_sum(e_lane), half_sum(g[0]), half_sum(g[1]), half_sum(g[2]));
    // torsion torques: prefix sums of (g, x cross g) within each half; the
    // half's last lane gives the torque about t
    float P[6];
    P[0] = g[0]; P[1] = g[1]; P[2] = g[2];
    P[3] = x[1] * g[2] - x[2] * g[1];
    P[4] = x[2] * g[0] - x[0] * g[2];
    P[5] = x[0] * g[1] - x[1] * g[0];
#pragma unroll
    for (int c = 0; c < 6; ++c) P[c] = half_scan(P[c]);
    const float4 TQ = make_float4(half_lane(P[3], kHalf - 1), half_lane(P[4], kHalf - 1),
                                  half_lane(P[5], kHalf - 1), 0.f);
    float gpsi = 0.f;
    {
        const int pk = j < L.T ? __float_as_int(sm.tor[j][0].w) : (1 << 16) | (1 << 24);
        const int t_apos = pk & 255, t_bpos = (pk >> 8) & 255;
        const int hi = ((pk >> 24) & 255) - 1, lo = ((pk >> 16) & 255) - 1;
        float S[6];
#pragma unroll
        for (int c = 0; c < 6; ++c)
            S[c] = __shfl(P[c], hb + (hi & (kHalf - 1))) - __shfl(P[c], hb + (lo & (kHalf - 1)));
        const float4 xa = dynh[t_apos & (kHalf - 1)];
        const float4 xb = dynh[t_bpos & (kHalf - 1)];
        float ux = xb.x - xa.x, uy = xb.y - xa.y, uz = xb.z - xa.z;
        const float il = __builtin_amdgcn_rsqf(ux * ux + uy * uy + uz * uz);
        ux *= il; uy *= il; uz *= il;
        const float mx = S[3] - (xa.y * S[2] - xa.z * S[1]);
        const float my = S[4] - (xa.z * S[0] - xa.x * S[2]);
        const float mz = S[5] - (xa.x * S[1] - xa.y * S[0]);
        gpsi = (j < L.T) ? ux * mx + uy * my + uz * mz : 0.f;
    }
    {
        const float k2 = 2.0f * qinv;
        const float gw = -(TQ.x * qx + TQ.y * qy + TQ.z * qz);
        const float gqx = qw * TQ.x + (TQ.y * qz - TQ.z * qy);
        const float gqy = qw * TQ.y + (TQ.z * qx - TQ.x * qz);
        const float gqz = qw * TQ.z + (TQ.x * qy - TQ.y * qx);
        const float gt = __shfl(gpsi, hb + ((j - 7) & (kHalf - 1)));
        float gr = gt;
        gr = j == 0 ? EG.y : gr;
        gr = j == 1 ? EG.z : gr;
        gr = j == 2 ? EG.w : gr;
        gr = j == 3 ? k2 * gw : gr;
        gr = j == 4 ? k2 * gqx : gr;
        gr = j == 5 ? k2 * gqy : gr;
        gr = j == 6 ? k2 * gqz : gr;
        grad = gr;
    }
    if (atom_out && j < N) {
        float4* o = reinterpret_cast<float4*>(atom_out) + 2 * L.orig[0];
        o[0] = make_float4(x[0], x[1], x[2], e_atom);
        o[1] = make_float4(g[0], g[1], g[2], 0.f);
    }
    return EG.x;
}

// ADADELTA local search of the two individuals ind0 and ind0 + 1 of an item
// (count = 1: only the first; the second half then mirrors the first and
// writes nothing). The steps are those of local_search_one.
template <bool ANY_LAYOUT>
__device__ void local_search_two(const DevItem& it, int ind0, int count, Smem2& sm, const Lig<1>& L,
                                 int iterations, float rho, float eps, bool final_eval) {
    const int lane = lane_id();
    const int j = lane & (kHalf - 1);
    const int h = lane >> 5;
    const bool live = h < count;
    const int ind = ind0 + (live ? h : 0);
    const int G = L.G;
    const bool act = j < G;
    const size_t o = (size_t)ind * G + j;
    float x = act ? it.genotype[o] : 0.f;
    float ag = act ? it.acc_g2[o] : 0.f;
    float ad = act ? it.acc_dx2[o] : 0.f;
    float bx = act ? it.best_genotype[o] : 0.f;
    float bestE = it.best_energy[ind];
    float lastE = it.energy[ind];
    float lastG = 0.f;
    for (int iter = 0; iter < iterations; ++iter) {
        float gr;
        const float E = evaluate2<ANY_LAYOUT>(it.grid, sm, L, x, gr, nullptr);
        lastE = E;
        lastG = gr;
        if (E < bestE) { bestE = E; bx = x; }
        gr = act ? gr : 0.f;
        ag = rho * ag + (1.f - rho) * gr * gr;
        const float dx = -(__builtin_amdgcn_sqrtf(ad + eps) * __builtin_amdgcn_rsqf(ag + eps)) * gr;
        ad = rho * ad + (1.f - rho) * dx * dx;
        float xn = x + dx;
        const bool isq = j >= 3 && j < 7;
        const float q2 = isq ? xn * xn : 0.f;
        const float nq2 = (half_lane(q2, 3) + half_lane(q2, 4)) + (half_lane(q2, 5) + half_lane(q2, 6));
        if (isq) xn = (nq2 >= 1e-12f) ? xn * __builtin_amdgcn_rsqf(nq2) : x;
        x = act ? xn : 0.f;
    }
    if (final_eval) {
        float gr;
        const float E = evaluate2<ANY_LAYOUT>(it.grid, sm, L, x, gr, nullptr);
        lastE = E;
        lastG = gr;
        if (E < bestE) { bestE = E; bx = x; }
    }
    if (!live) return;
    if (act && it.grad && (iterations > 0 || final_eval)) it.grad[o] = lastG;
    if (act) {
        it.genotype[o] = x;
        it.acc_g2[o] = ag;
        it.acc_dx2[o] = ad;
        it.best_genotype[o] = bx;
    }
    if (j == 0) {
        it.best_energy[ind] = bestE;
        it.energy[ind] = lastE;
        it.iters_done[ind] += iterations;
    }
}

// Persistent local-search kernel, two individuals per wave: work units are
// pairs of individuals of one item ((n + 1) / 2 per item), pulled from the
// counter as in ls_kernel.
template <bool ANY_LAYOUT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 3))) void ls_kernel_two(LsParams p) {
    __shared__ Smem2 sm;
    int cur_item = -1;
    while (true) {
        int u = 0;
        if (lane_id() == 0) u = atomicAdd(p.counter, 1);
        u = uniform(u);
        if (u >= p.total_units) break;
        const int lo = item_of_unit(p, u);
        const DevItem it = load_item(p.items, lo);
        const int ind0 = 2 * (u - it.unit_begin);
        const int count = min(2, it.n - ind0);
        const bool reload = lo != cur_item;
        cur_item = lo;
        Lig<1> L;
        load_ligand2(it.blob, sm, L, reload);
        local_search_two<ANY_LAYOUT>(it, ind0, count, sm, L, it.iterations, p.rho, p.eps, it.final_eval != 0);
    }
}

// One persistent launch for a batch that mixes two-wave individuals with
// one-wave units (an individual of a ligand of <= 64 atoms, or a pair of
// individuals two per wave): 128-thread blocks, two work counters. Units
// [0, block_units) are the two-wave individuals (their items come first):
// a block takes them from the first counter as ls_kernel_mw does. Once that
// counter passes them, or from the start for the last wave_blocks blocks of
// the grid, each wave takes the remaining units from the second counter on
// its own, in its own half of the block's LDS, ordering its LDS accesses at
// wave scope only (the other wave may be anywhere in its own unit). Every
// wave exits once the second counter passes the last unit.
constexpr size_t kWaveLds =
    ((sizeof(Smem2) > sizeof(Smem<1>) ? sizeof(Smem2) : sizeof(Smem<1>)) + 15) / 16 * 16;

struct __align__(16) SmemUni {
    union {
        Smem<1, 2> two;                       // a two-wave individual
        unsigned char wave[2][kWaveLds];      // per wave: Smem<1> or Smem2
    } u;
    int unit;                                 // outside the union: read after the
                                              // waves start writing their halves
};
static_assert(sizeof(SmemUni) <= 20 * 1280, "six 128-thread blocks per CU");

template <int VAR>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(3, 3))) void ls_kernel_uni(LsParams p) {
    __shared__ SmemUni sm;
    int cur_item = -1;
    if ((int)blockIdx.x < (int)gridDim.x - p.wave_blocks) {
        while (true) {
            __syncthreads();                   // the previous unit is read by both waves
            if (threadIdx.x == 0) sm.unit = atomicAdd(p.counter, 1);
            __syncthreads();
            const int u = uniform(sm.unit);
            if (u >= p.block_units) break;
            const int lo = item_of_unit(p, u);
            const DevItem it = load_item(p.items, lo);
            const bool reload = lo != cur_item;
            cur_item = lo;
            Lig<1> L;
            load_ligand<1, 2>(it.blob, sm.u.two, L, reload);
            ls_run<1, VAR, 2>(it, u - it.unit_begin, sm.u.two, L, p);
        }
    }
    const int w = uniform((int)threadIdx.x >> 6);
    unsigned char* const lds = sm.u.wave[w];
    cur_item = -1;                             // the two-wave tables are gone
    while (true) {
        int v = 0;
        if (lane_id() == 0) v = atomicAdd(p.counter2, 1);
        const int next = p.block_units + uniform(v);
        if (next >= p.total_units) break;
        const int lo = item_of_unit(p, next);
        const DevItem it = load_item(p.items, lo);
        const bool reload = lo != cur_item;
        cur_item = lo;
        Lig<1> L;
        if (it.pack == 2) {
            Smem2& s2 = *reinterpret_cast<Smem2*>(lds);
            const int ind0 = 2 * (next - it.unit_begin);
            load_ligand2(it.blob, s2, L, reload);
            local_search_two<false>(it, ind0, min(2, it.n - ind0), s2, L, it.iterations, p.rho, p.eps,
                                    it.final_eval != 0);
        } else {
            Smem<1>& s1 = *reinterpret_cast<Smem<1>*>(lds);
            load_ligand<1, 1>(it.blob, s1, L, reload);
            ls_run<1, VAR, 1>(it, next - it.unit_begin, s1, L, p);
        }
    }
}

// Persistent scoring kernel, two genotypes per wave (ind = 2 k + half).
template <bool ANY_LAYOUT>
__global__ __launch_bounds__(64, 3) void score_kernel_two(GridParams G, const uint8_t* __restrict__ blob, int n,
                                                          const float* __restrict__ gen,
                                                          float* __restrict__ energy,
                                                          float* __restrict__ grad,
                                                          float* __restrict__ atom_out) {
    __shared__ Smem2 sm;
    Lig<1> L;
    load_ligand2(blob, sm, L);
    const int lane = lane_id();
    const int j = lane & (kHalf - 1);
    const int h = lane >> 5;
    const int G_ = L.G;
    const int n_pairs = (n + 1) >> 1;
    for (int k = blockIdx.x; k < n_pairs; k += gridDim.x) {
        const bool live = 2 * k + h < n;
        const int ind = live ? 2 * k + h : 2 * k;
        const float gene = j < G_ ? gen[(size_t)ind * G_ + j] : 0.f;
        float gr;
        float* ao = (atom_out && live) ? atom_out + (size_t)ind * L.N * 8 : nullptr;
        const float E = evaluate2<ANY_LAYOUT>(G, sm, L, gene, gr, ao);
        if (live && j == 0) energy[ind] = E;
        if (live && grad && j < G_) grad[(size_t)ind * G_ + j] = gr;
    }
}

// Sum over the first 16-lane row (lanes 16..63 ignored), every lane receives it.
__device__ __forceinline__ float row0_sum(float v) {
    v += dpp<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);   // row_half_mirror
    v += dpp<0x140>(v);   // row_mirror
    return readlane(v, 0);
}

// Isolated block sum (reduction test kernel): every thread holds a float4;
// each wave reduces with the chosen variant, the per-wave totals (at most 16)
// meet in LDS after one barrier, and every wave adds them with a butterfly
// over its first row (lane l holds wave l's total), so every thread gets the
// block total in a fixed order.
template <int VAR>
__global__ __launch_bounds__(1024) void block_sum4_kernel(const float4* __restrict__ in,
                                                          float4* __restrict__ out, int repeat,
                                                          float chain) {
    __shared__ float4 part[2][16];
    const int t = threadIdx.x;
    const int nw = blockDim.x >> 6;
    const int w = t >> 6;
    const int lane = t & 63;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + t;
    const float4 v0 = in[idx];
    float4 v = v0;
    float4 tot = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int r = 0; r < repeat; ++r) {
        const float4 ws = sum4<VAR>(v);
        if (nw == 1) {
            tot = ws;
        } else {
            if (lane == 0) part[r & 1][w] = ws;
            __syncthreads();
            const float4 p = lane < nw ? part[r & 1][lane & 15] : make_float4(0.f, 0.f, 0.f, 0.f);
            tot = make_float4(row0_sum(p.x), row0_sum(p.y), row0_sum(p.z), row0_sum(p.w));
        }
        v = make_float4(v0.x + chain * tot.x, v0.y + chain * tot.y, v0.z + chain * tot.z,
                        v0.w + chain * tot.w);
    }
    out[idx] = tot;
}

// The Sec. 3 baseline, for the reduction test only: per component, a wave
// shuffle tree, then the first lane of each wave adds its value into a
// shared accumulator with an atomic, a barrier, and every thread reads the
// accumulator back (three barriers per component, as described there).
__global__ __launch_bounds__(1024) void block_sum4_atomic_kernel(const float4* __restrict__ in,
                                                                 float4* __restrict__ out,
                                                                 int repeat, float chain) {
    __shared__ float acc[4];
    const int t = threadIdx.x;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + t;
    const float4 v0 = in[idx];
    float4 v = v0;
    float4 tot = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int r = 0; r < repeat; ++r) {
        float vc[4] = {v.x, v.y, v.z, v.w};
        float res[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (t == 0) acc[c] = 0.f;
            __syncthreads();
            float s = vc[c];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
            if ((t & 63) == 0) atomicAdd(&acc[c], s);
            __syncthreads();
            res[c] = acc[c];
            __syncthreads();
        }
        tot = make_float4(res[0], res[1], res[2], res[3]);
        v = make_float4(v0.x + chain * tot.x, v0.y + chain * tot.y, v0.z + chain * tot.z,
                        v0.w + chain * tot.w);
    }
    out[idx] = tot;
}

template <int SLOTS, int VAR, bool ANY>
hipError_t launch_score_k(const GridParams& g, const uint8_t* blob, int n, const float* gen, float* energy,
                          float* grad, float* atom_out, int n_cu, hipStream_t st) {
    auto k = score_kernel<SLOTS, VAR, ANY>;
    // resident blocks per CU, queried once per kernel (the query costs tens
    // of microseconds of host time, as much as a small call's kernel)
    static std::atomic<int> cached{0};
    int per_cu = cached.load(std::memory_order_relaxed);
    if (per_cu <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k), 64, 0) !=
                hipSuccess ||
            per_cu <= 0)
            per_cu = 2;
        cached.store(per_cu, std::memory_order_relaxed);
    }
    const long long resident = (long long)per_cu * (n_cu > 0 ? n_cu : 256);
    const int blocks = (int)(n < resident ? n : resident);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64), 0, st, g, blob, n, gen, energy, grad, atom_out);
    return hipGetLastError();
}

template <int VAR>
hipError_t launch_score_v(const GridParams& g, const uint8_t* blob, int slots, int n,
                          const float* gen, float* energy, float* grad, float* atom_out, int n_cu,
                          hipStream_t st) {
    const bool any = g.corners == nullptr;
    if (slots == 1)
        return any ? launch_score_k<1, VAR, true>(g, blob, n, gen, energy, grad, atom_out, n_cu, st)
                   : launch_score_k<1, VAR, false>(g, blob, n, gen, energy, grad, atom_out, n_cu, st);
    return any ? launch_score_k<2, VAR, true>(g, blob, n, gen, energy, grad, atom_out, n_cu, st)
               : launch_score_k<2, VAR, false>(g, blob, n, gen, energy, grad, atom_out, n_cu, st);
}

template <int VAR>
hipError_t launch_sw_v(const GridParams& g, const uint8_t* blob, int slots, const docklaunch::SwParams& p,
                       hipStream_t st) {
    if (slots == 1)
        hipLaunchKernelGGL((sw_kernel<1, VAR>), dim3(p.n), dim3(64), 0, st, g, blob, p);
    else
        hipLaunchKernelGGL((sw_kernel<2, VAR>), dim3(p.n), dim3(64), 0, st, g, blob, p);
    return hipGetLastError();
}

template <int MODE>
const void* ls_kernel_ptr(int var) {
    switch (var) {
        case 0: return reinterpret_cast<const void*>(&ls_kernel<MODE, 0>);
        case 1: return reinterpret_cast<const void*>(&ls_kernel<MODE, 1>);
        case 2: return reinterpret_cast<const void*>(&ls_kernel<MODE, 2>);
        case 3: return reinterpret_cast<const void*>(&ls_kernel<MODE, 3>);
        case 4: return reinterpret_cast<const void*>(&ls_kernel<MODE, 4>);
        default: return reinterpret_cast<const void*>(&ls_kernel<MODE, -1>);
    }
}

template <int WAVES>
const void* ls_kernel_mw_ptr(int var) {
    switch (var) {
        case 0: return reinterpret_cast<const void*>(&ls_kernel_mw<0, WAVES>);
        case 1: return reinterpret_cast<const void*>(&ls_kernel_mw<1, WAVES>);
        case 2: return reinterpret_cast<const void*>(&ls_kernel_mw<2, WAVES>);
        case 3: return reinterpret_cast<const void*>(&ls_kernel_mw<3, WAVES>);
        case 4: return reinterpret_cast<const void*>(&ls_kernel_mw<4, WAVES>);
        default: return reinterpret_cast<const void*>(&ls_kernel_mw<-1, WAVES>);
    }
}

const void* ls_kernel_uni_ptr(int var) {
    switch (var) {
        case 0: return reinterpret_cast<const void*>(&ls_kernel_uni<0>);
        case 1: return reinterpret_cast<const void*>(&ls_kernel_uni<1>);
        case 2: return reinterpret_cast<const void*>(&ls_kernel_uni<2>);
        case 3: return reinterpret_cast<const void*>(&ls_kernel_uni<3>);
        case 4: return reinterpret_cast<const void*>(&ls_kernel_uni<4>);
        default: return nullptr;             // the plan gives this launch one variant
    }
}

const void* ls_kernel_for(int mode, int var) {
    if (mode == docklaunch::kTwoPerWave)
        return var == DOCK_REDUCE_SHUFFLE ? reinterpret_cast<const void*>(&ls_kernel_two<false>)
                                          : reinterpret_cast<const void*>(&ls_kernel_two<true>);
    if (mode == docklaunch::kTwoWave) return ls_kernel_mw_ptr<2>(var);
    if (mode == docklaunch::kFourWave) return ls_kernel_mw_ptr<4>(var);
    if (mode == docklaunch::kUnified) return ls_kernel_uni_ptr(var);
    if (mode == docklaunch::kSlots1) return ls_kernel_ptr<docklaunch::kSlots1>(var);
    if (mode == docklaunch::kSlots2) return ls_kernel_ptr<docklaunch::kSlots2>(var);
    return ls_kernel_ptr<docklaunch::kSlotsAny>(var);
}

}  // namespace

namespace docklaunch {

hipError_t launch_score(const GridParams& g, const uint8_t* blob, int slots, int n,
                        const float* genotypes, float* energy, float* grad, float* atom_out,
                        int variant, int n_cu, hipStream_t stream) {
    switch (variant) {
        case DOCK_REDUCE_SHUFFLE: return launch_score_v<0>(g, blob, slots, n, genotypes, energy, grad, atom_out, n_cu, stream);
        case DOCK_REDUCE_MFMA_F32: return launch_score_v<1>(g, blob, slots, n, genotypes, energy, grad, atom_out, n_cu, stream);
        case DOCK_REDUCE_MFMA_BF16: return launch_score_v<2>(g, blob, slots, n, genotypes, energy, grad, atom_out, n_cu, stream);
        case DOCK_REDUCE_MFMA_F16: return launch_score_v<3>(g, blob, slots, n, genotypes, energy, grad, atom_out, n_cu, stream);
        case DOCK_REDUCE_MFMA_BF16X3: return launch_score_v<4>(g, blob, slots, n, genotypes, energy, grad, atom_out, n_cu, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_score_two(const GridParams& g, const uint8_t* blob, int n, const float* genotypes,
                            float* energy, float* grad, float* atom_out, int n_cu, hipStream_t stream) {
    const bool any = g.corners == nullptr;
    const void* k = any ? reinterpret_cast<const void*>(&score_kernel_two<true>)
                        : reinterpret_cast<const void*>(&score_kernel_two<false>);
    static std::atomic<int> cached[2];
    int per_cu = cached[any ? 1 : 0].load(std::memory_order_relaxed);
    if (per_cu <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 64, 0) != hipSuccess || per_cu <= 0) per_cu = 2;
        cached[any ? 1 : 0].store(per_cu, std::memory_order_relaxed);
    }
    const long long pairs = ((long long)n + 1) / 2;
    const long long resident = (long long)per_cu * (n_cu > 0 ? n_cu : 256);
    const int blocks = (int)(pairs < resident ? pairs : resident);
    GridParams gg = g;
    const uint8_t* bb = blob;
    int nn = n;
    const float* gen = genotypes;
    float* e = energy;
    float* gr = grad;
    float* ao = atom_out;
    void* args[] = {&gg, &bb, &nn, &gen, &e, &gr, &ao};
    return hipLaunchKernel(k, dim3(blocks), dim3(64), args, 0, stream);
}

hipError_t launch_sw(const GridParams& g, const uint8_t* blob, int slots, int variant, const SwParams& p,
                     hipStream_t stream) {
    switch (variant) {
        case DOCK_REDUCE_SHUFFLE: return launch_sw_v<0>(g, blob, slots, p, stream);
        case DOCK_REDUCE_MFMA_F32: return launch_sw_v<1>(g, blob, slots, p, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_expand_corners(const GridParams& g, float* corners, hipStream_t stream) {
    const long long total = (long long)(g.n_maps - 2) * (g.nx - 1) * (g.ny - 1) * (g.nz - 1);
    if (total <= 0) return hipSuccess;
    const long long blocks = (total + 255) / 256;
    hipLaunchKernelGGL(expand_corners_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, g,
                       reinterpret_cast<float4*>(corners), total);
    return hipGetLastError();
}

hipError_t launch_ls(const LsParams& p, int mode, int variant_uniform, int grid_blocks,
                     hipStream_t stream) {
    const void* k = ls_kernel_for(mode, variant_uniform);
    if (!k) return hipErrorInvalidValue;
    LsParams pp = p;
    void* args[] = {&pp};
    return hipLaunchKernel(k, dim3(grid_blocks), dim3(ls_block_threads(mode)), args, 0, stream);
}

int ls_blocks_per_cu(int mode, int variant_uniform) {
    // cached per (mode, variant): the occupancy query costs host time on
    // every call otherwise
    static std::atomic<int> cache[docklaunch::kLsModes][DOCK_REDUCE_COUNT + 1];
    const int m = mode >= 0 && mode < docklaunch::kLsModes ? mode : 0;
    const int v = variant_uniform >= 0 && variant_uniform < DOCK_REDUCE_COUNT ? variant_uniform : DOCK_REDUCE_COUNT;
    int nb = cache[m][v].load(std::memory_order_relaxed);
    if (nb > 0) return nb;
    const void* k = ls_kernel_for(mode, variant_uniform);
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, ls_block_threads(mode), 0) != hipSuccess) return 0;
    cache[m][v].store(nb, std::memory_order_relaxed);
    return nb;
}

hipError_t launch_block_sum4(const float* in, float* out, int n_blocks, int threads, int variant,
                             int repeat, hipStream_t stream) {
    const float4* i4 = reinterpret_cast<const float4*>(in);
    float4* o4 = reinterpret_cast<float4*>(out);
    const float chain = 0.0f;
    switch (variant) {
        case 0: hipLaunchKernelGGL((block_sum4_kernel<0>), dim3(n_blocks), dim3(threads), 0, stream, i4, o4, repeat, chain); break;
        case 1: hipLaunchKernelGGL((block_sum4_kernel<1>), dim3(n_blocks), dim3(threads), 0, stream, i4, o4, repeat, chain); break;
        case 2: hipLaunchKernelGGL((block_sum4_kernel<2>), dim3(n_blocks), dim3(threads), 0, stream, i4, o4, repeat, chain); break;
        case 3: hipLaunchKernelGGL((block_sum4_kernel<3>), dim3(n_blocks), dim3(threads), 0, stream, i4, o4, repeat, chain); break;
        case 4: hipLaunchKernelGGL((block_sum4_kernel<4>), dim3(n_blocks), dim3(threads), 0, stream, i4, o4, repeat, chain); break;
        case 5: hipLaunchKernelGGL(block_sum4_atomic_kernel, dim3(n_blocks), dim3(threads), 0, stream, i4, o4, repeat, chain); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace docklaunch
