// Internal interface between the C ABI (dock_abi.cpp) and the kernels
// (dock_kernels.hip). Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace docklaunch {

// Receptor grid as the kernels see it.
struct GridParams {
    const float* maps;   // [n_maps][nz][ny][nx]
    const float* corners;  // nullptr, or per atom type and cell the cell's 8 corner values
                           // v[4 dz + 2 dy + dx] of the type map, the electrostatic and
                           // the desolvation map, padded to 128 bytes:
                           // [n_maps-2][(nz-1)(ny-1)(nx-1)][32] (24 values, 8 zeros)
    int32_t nx, ny, nz, n_maps;
    float spacing;
    float inv_spacing;
    float origin[3];
    float hi[3];         // origin + (n - 1) * spacing per axis
};

// One local-search item as the kernels see it (lives in the workspace).
struct DevItem {
    GridParams grid;
    const uint8_t* blob;
    float* genotype;
    float* acc_g2;
    float* acc_dx2;
    float* best_genotype;
    float* best_energy;
    float* energy;
    int32_t* iters_done;
    float* grad;            // optional: gradient at the last evaluated point
    int32_t n;
    int32_t variant;
    int32_t slots;          // 1 if n_atoms <= 64, else 2
    int32_t unit_begin;     // first work unit (individual) of this item
    int32_t iterations;     // steps for this item
    int32_t final_eval;     // evaluate the point reached after the last step
    int32_t pack;           // individuals per wave: 2 (two per wave), else 1
    int32_t pad_;
};

struct LsParams {
    const DevItem* items;   // device
    int32_t* counter;       // device, zero at launch
    int32_t* counter2;      // one mixed launch: the one-wave units' counter, zero at launch
    int32_t n_items;
    int32_t total_units;
    int32_t block_units;    // one mixed launch: units [0, block_units) take both waves of a block
    int32_t wave_blocks;    // one mixed launch: the last wave_blocks blocks take one-wave units only
    float rho, eps;
};

// Workspace layout: [int32 work counters (one per launch of a call, and at
// index 8 + k the second counter of a shared launch k), 64 B][DevItem x n_items]
constexpr int64_t kWorkspaceHeader = 64;

// ls kernel families: slots 1, slots 2, or both (runtime per item), all one
// wave per individual; two or four waves per individual; two individuals
// per wave (ligands of <= 32 atoms and <= 32 genes, shuffle reduction); or
// one launch holding two-wave individuals, one-slot individuals and pairs
// two per wave (one variant, corner-expanded maps)
enum LsMode { kSlots1 = 1, kSlots2 = 2, kSlotsAny = 3, kTwoWave = 4, kTwoPerWave = 5, kFourWave = 6,
              kUnified = 7 };
constexpr int kLsModes = 8;

inline int ls_block_threads(int mode) {
    return (mode == kTwoWave || mode == kUnified) ? 128 : (mode == kFourWave ? 256 : 64);
}

// Persistent: at most the resident blocks of n_cu CUs, each looping over
// genotypes with a stride of the grid size.
hipError_t launch_score(const GridParams& g, const uint8_t* blob, int slots, int n,
                        const float* genotypes, float* energy, float* grad, float* atom_out,
                        int variant, int n_cu, hipStream_t stream);
// Two genotypes per wave (ligands of <= 32 atoms and <= 32 genes; the
// shuffle reduction).
hipError_t launch_score_two(const GridParams& g, const uint8_t* blob, int n, const float* genotypes,
                            float* energy, float* grad, float* atom_out, int n_cu, hipStream_t stream);

// variant_uniform: DOCK_REDUCE_* when every item uses it, -1 for mixed items.
hipError_t launch_ls(const LsParams& p, int mode, int variant_uniform, int grid_blocks,
                     hipStream_t stream);

// Resident blocks per CU for the ls kernel family chosen by
// (mode, variant_uniform); 0 on error.
int ls_blocks_per_cu(int mode, int variant_uniform);

hipError_t launch_block_sum4(const float* in, float* out, int n_blocks, int threads,
                             int variant, int repeat, hipStream_t stream);

// Writes the corner-expanded copy of g.maps (layout of GridParams::corners).
hipError_t launch_expand_corners(const GridParams& g, float* corners, hipStream_t stream);

// Solis-Wets search state and draws (dock_solis_wets_batch), one individual per block.
struct SwParams {
    const float* normals;     // [iterations][n][G] standard normal draws
    const float* scale;       // [G] per-gene step scale
    float* genotype;          // [n][G] in/out
    float* energy;            // [n] in/out: energy of genotype
    float* bias;              // [n][G] in/out
    float* rho;               // [n] in/out
    int32_t* counts;          // [n][2] in/out: successes, failures in a row
    float* log;               // optional [n][iterations][2]: the trials' energies (NaN: not tried)
    int32_t n, iterations, n_success, n_failure;
};

// variant: DOCK_REDUCE_SHUFFLE or DOCK_REDUCE_MFMA_F32.
hipError_t launch_sw(const GridParams& g, const uint8_t* blob, int slots, int variant, const SwParams& p,
                     hipStream_t stream);

// One GA generation step (the operators of dock_ga_step).
struct GaParams {
    const float* genotypes;   // [n_runs][pop][n_genes]
    const float* energies;    // [n_runs][pop]
    const int32_t* cand;      // [n_runs][pop][4]
    const float* coins;       // [n_runs][pop][3]
    const int32_t* cuts;      // [n_runs][pop][2]
    const float* mut_coin;    // [n_runs][pop][n_genes]
    const float* mut_delta;   // [n_runs][pop][n_genes]
    float* children;          // [n_runs][pop][n_genes]
    int32_t* best;            // [n_runs]
    int32_t n_runs, pop, n_genes;
    float p_tournament, p_crossover, p_mutation;
    int32_t elitism;
};

hipError_t launch_ga_step(const GaParams& p, hipStream_t stream);

// Rows with draws[r] < rate, in increasing order, and their count (one block).
hipError_t launch_select_rows(const float* draws, int n, float rate, int32_t* index, int32_t* count,
                              hipStream_t stream);
// Gather (dst[k] = src[index[k]]) or scatter (dst[index[k]] = src[k]) of m
// rows of `row` floats; n_rows bounds the indexed side.
hipError_t launch_move_rows(bool gather, const float* src, float* dst, const int32_t* index, int m, int row,
                            int n_rows, hipStream_t stream);

// Library-resident workspace (dock_local_search_batch_static): its size in
// bytes, and its device address on the current device (looked up once per
// device with hipGetSymbolAddress).
int64_t static_workspace_capacity();
hipError_t static_workspace(void** out);

// Writes `bytes` (a multiple of 4) of host memory to dst_dev on `stream` by
// kernel launches that carry the data in their arguments (no host staging,
// no copy or memset node).
hipError_t launch_table_fill(void* dst_dev, const void* src_host, int64_t bytes, hipStream_t stream);

}  // namespace docklaunch
