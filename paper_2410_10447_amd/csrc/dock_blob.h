// Packed device layout of a prepared ligand, shared by the host preparation
// (dock_host.cpp) and the kernels (dock_kernels.hip).
//
// Atoms are stored in depth-first order from the root atom, so the atoms a
// torsion moves form one contiguous range [first, end) of positions. All
// sections start on a 16-byte boundary; offsets are in bytes from the blob
// start.
//
// Intramolecular pairs are not stored as a list. A lane that owns atom a
// visits partner b = (a + s) mod N for s = 1 .. N/2 (a circulant schedule that
// meets every unordered pair exactly once, the middle step of an even N only
// from a < N/2), and three per-atom 64-bit masks say, for each step s (bit
// s-1), whether the pair is kept, whether it is a hydrogen-bond pair, and the
// partner's donor/acceptor index. Pair parameters are rebuilt from per-atom
// values: r0 = R_a + R_b, eps = sqrt(eps_a) sqrt(eps_b), 332.06363 q_a q_b,
// S_a V_b + S_b V_a, or the 12-10 table entry of the donor-acceptor pair.
#pragma once
#include <stdint.h>

namespace dockblob {

constexpr int32_t kMagic = 0x444f434b;  // "DOCK"
constexpr int kMaxAtoms = 128;
constexpr int kMaxTorsions = 32;
constexpr int kMaxFrag = kMaxTorsions + 1;
constexpr int kChainStride = kMaxTorsions + 1;  // [0] = length, [1..] torsion ids root first

struct Header {
    int32_t magic;
    int32_t n_atoms;
    int32_t n_torsions;
    int32_t n_frag;
    int32_t n_genes;
    int32_t n_pairs;
    int32_t max_depth;
    int32_t n_steps;        // floor(n_atoms / 2)
    int32_t max_class;      // largest atom class used (type-map index)
    int32_t total_bytes;
    // section offsets (bytes)
    int32_t off_ref;        // float4[N]  y0 (reference coords minus centroid), w = 0
    int32_t off_par;        // float4[N]  R, sqrt(eps), S = s + 0.01097|q|, V
    int32_t off_chg;        // float4[N]  332.06363 q, q, |q|, 0
    int32_t off_hb;         // float4[N]  12-10 r0 vs partner index 0/1, eps vs 0/1
    int32_t off_int;        // int4[N]    class, fragment, original index, 0
    int32_t off_mask;       // uint64[3][N] kept / hb / partner hb index, bit s-1
    int32_t off_tors;       // Torsion[T]
    int32_t off_chain;      // int8[n_frag][kChainStride]
    int32_t pad[14];
};
static_assert(sizeof(Header) == 128, "header is 128 bytes");

struct Torsion {
    float p[4];      // axis point y0[a] (w unused)
    float u[4];      // unit axis y0[b] - y0[a] (w unused)
    int32_t a_pos, b_pos, first, end;  // depth-first positions; moving range [first, end)
};
static_assert(sizeof(Torsion) == 48, "torsion record is 48 bytes");

}  // namespace dockblob
