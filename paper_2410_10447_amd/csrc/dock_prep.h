// Host-side ligand preparation: depth-first order, torsion ranges, rigid
// fragments, pair masks and the packed device blob. Plain C++ (no HIP), so
// it can be built and checked on a machine without a GPU.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "dock.h"
#include "dock_blob.h"

namespace dockprep {

struct Prepared {
    int n_atoms = 0, n_torsions = 0, n_frag = 0, max_depth = 0, n_pairs = 0, max_class = 0;
    std::vector<int32_t> order;        // depth-first position -> original atom
    std::vector<int32_t> pos;          // original atom -> depth-first position
    std::vector<int32_t> tors_a, tors_b;       // original indices, a on the root side
    std::vector<int32_t> tors_first, tors_end; // moving range of positions
    std::vector<int32_t> frag_of_atom;         // original index -> fragment id
    std::vector<uint8_t> blob;                 // packed device layout (dockblob)
};

// Returns DOCK_OK or an error status with `err` set.
int32_t prepare(const dock_ligand_desc& d, Prepared& out, std::string& err);

// Pairs decoded from the blob's masks: (i << 16) | j, i < j original, sorted.
void decode_pairs(const Prepared& p, std::vector<uint32_t>& pairs, std::vector<uint8_t>& hb);
// Record k of the packed pair list, in the logical layout (dockblob).
uint32_t record_of(const Prepared& p, int k);

}  // namespace dockprep
