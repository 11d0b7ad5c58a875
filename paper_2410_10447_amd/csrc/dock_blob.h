// Packed device layout of a prepared ligand, shared by the host preparation
// (dock_prep.cpp) and the kernels (dock_kernels.hip).
//
// Atoms are stored in depth-first order from the root atom, so the atoms a
// torsion moves form one contiguous range [first, end) of positions. All
// sections start on a 16-byte boundary; offsets are in bytes from the blob
// start.
//
// Intramolecular pairs are stored as a list cut into batches of 64, one pair
// per lane. Within a batch an atom appears at most n_copies times, and each
// appearance is given its own copy index, so the force updates of one batch
// go to distinct accumulator slots (copy * slot_stride + atom, slot_stride the
// smallest power of two >= max(n_atoms, 16)): a lane can add its pair's force
// to both atoms without two lanes of one instruction touching the same
// address, and the order of additions is fixed by the list. Each pair
// carries its own parameters, computed on the host in double precision and
// rounded once: the dispersion-repulsion coefficients A, B of A / r^12 +
// B / r^m (from r0 = R_a + R_b and eps = sqrt(eps_a eps_b), or the 12-10
// table entry of the donor-acceptor pair) and the desolvation weight
// S_a V_b + S_b V_a. The Coulomb factor q_a q_b comes from the charges the
// kernel keeps with the atom positions.
#pragma once
#include <stdint.h>

namespace dockblob {

constexpr int32_t kMagic = 0x444f434b;  // "DOCK"
constexpr int kMaxAtoms = 128;
constexpr int kMaxTorsions = 32;
constexpr int kMaxFrag = kMaxTorsions + 1;
constexpr int kChainStride = kMaxTorsions;      // torsion ids innermost first, padded with
constexpr int kIdentity = kMaxTorsions;          // kIdentity (the identity transform)
constexpr int kBatch = 64;
constexpr int kMaxSlots = 384;                   // n_copies * slot_stride <= kMaxSlots
constexpr int kMaxSlotsSmall = 320;              // the same bound for ligands of <= 64 atoms
constexpr int kMaxSlotsTiny = 288;               // and for ligands of <= 32 atoms

// Accumulator (and position) stride: the smallest power of two >= n_atoms,
// at least 16. Slots of "atoms" n_atoms .. stride-1 are never summed; unused
// lanes may write there.
inline int slot_stride(int n_atoms) {
    int s = 16;
    while (s < n_atoms) s <<= 1;
    return s;
}

// Logical pair record (host side, and the batches the library exports):
// i | j << 7 | ci << 14 | cj << 18 | hb << 22 | table << 23 | valid << 31
// (table: index 2 * donor + acceptor of a 12-10 pair's parameters)
constexpr uint32_t kRecValid = 1u << 31;
inline uint32_t make_record(int i, int j, int ci, int cj, int hb, int table) {
    return (uint32_t)i | ((uint32_t)j << 7) | ((uint32_t)ci << 14) | ((uint32_t)cj << 18) |
           ((uint32_t)hb << 22) | ((uint32_t)table << 23) | kRecValid;
}
// An unused lane: valid bit clear, two distinct slots no pair of the batch uses.
inline uint32_t make_pad_record(int i, int j, int ci, int cj) {
    return (uint32_t)i | ((uint32_t)j << 7) | ((uint32_t)ci << 14) | ((uint32_t)cj << 18);
}

// Device record word: the byte offsets (copy * stride + atom) * 16 of the two
// accumulator slots in bits 0..12 and 13..25, the 12-10 flag in bit 31. An
// atom's position lies at its slot offset masked with stride * 16 - 1. An
// unused lane has c12 = -0.0f (its bit pattern kPadC12), A = B = ds = 0.
constexpr int kSlotShift = 13;
constexpr uint32_t kSlotMask = (1u << kSlotShift) - 1;
constexpr uint32_t kDevHb = 1u << 31;
constexpr uint32_t kPadC12 = 0x80000000u;
static_assert(kMaxSlots * 16 <= (int)kSlotMask + 1, "slot byte offsets fit 13 bits");
inline uint32_t device_word(uint32_t logical, int stride) {
    const uint32_t i = logical & 127, j = (logical >> 7) & 127;
    const uint32_t ci = (logical >> 14) & 15, cj = (logical >> 18) & 15;
    const uint32_t hb = (logical & kRecValid) ? (logical >> 22) & 1 : 0;
    return ((ci * stride + i) << 4) | (((cj * stride + j) << 4) << kSlotShift) | (hb ? kDevHb : 0u);
}
// The logical record of a device word (table index not kept: 0).
inline uint32_t logical_record(uint32_t word, bool valid, int stride) {
    const uint32_t si = (word & kSlotMask) >> 4, sj = ((word >> kSlotShift) & kSlotMask) >> 4;
    const uint32_t s = (uint32_t)stride;
    const uint32_t rec = (si % s) | ((sj % s) << 7) | ((si / s) << 14) | ((sj / s) << 18);
    return valid ? rec | (((word & kDevHb) ? 1u : 0u) << 22) | kRecValid : rec;
}

struct Header {
    int32_t magic;
    int32_t n_atoms;
    int32_t n_torsions;
    int32_t n_frag;
    int32_t n_genes;
    int32_t n_pairs;
    int32_t max_depth;
    int32_t n_batches;      // pair batches of kBatch records
    int32_t n_copies;       // accumulator copies per atom
    int32_t max_class;      // largest atom class used (type-map index)
    int32_t total_bytes;
    // section offsets (bytes)
    int32_t off_ref;        // float4[N]  y0 (reference coords minus centroid), w = 0
    int32_t off_chg;        // float4[N]  332.06363 q, q, |q|, 0
    int32_t off_int;        // int4[N]    class, fragment, original index, 0
    int32_t off_tors;       // Torsion[T]
    int32_t off_chain;      // uint8[n_frag][kChainStride] enclosing torsions, innermost first
    int32_t off_plist;      // PairRec[n_batches][kBatch]
    int32_t slot_stride;    // accumulator stride, see slot_stride()
    int32_t pad[14];
};
static_assert(sizeof(Header) == 128, "header is 128 bytes");

// One lane's pair: the device record word, then A = eps a r0^12,
// B = eps b r0^m (12-6: a = 1, b = -2, m = 6; 12-10: a = 5, b = -6, m = 10)
// and the desolvation weight; an unused lane has A = -0.0f, B = ds = 0.
struct PairRec {
    uint32_t rec;
    float c12, cm, ds;
};
static_assert(sizeof(PairRec) == 16, "pair record is 16 bytes");

struct Torsion {
    float p[4];      // axis point y0[a] (w unused)
    float u[4];      // unit axis y0[b] - y0[a] (w unused)
    int32_t a_pos, b_pos, first, end;  // depth-first positions; moving range [first, end)
};
static_assert(sizeof(Torsion) == 48, "torsion record is 48 bytes");

}  // namespace dockblob
