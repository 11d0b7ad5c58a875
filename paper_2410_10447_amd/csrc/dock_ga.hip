// GA generation step of the LGA (Sec. 2.1 names the genetic search; the
// operators are the standard AutoDock ones, see dock_ga_step in dock.h):
// the best member of each run, then one thread per child gene.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dock_launch.h"

namespace {

// ---------------------------------------------------------------------------
// GA generation step (the genetic half of the LGA, Sec. 2.1): elitism,
// binary tournaments, two-point crossover, additive mutation; every random
// number is an input. Energies rank with NaN as +inf.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float ga_key(float e) { return __builtin_isnan(e) ? __builtin_inff() : e; }

// (key, index) pairs ordered by key, then index: the first of the minima.
__device__ __forceinline__ void ga_min(float& k, int& i, float k2, int i2) {
    if (k2 < k || (k2 == k && i2 < i)) { k = k2; i = i2; }
}

// Best member of run blockIdx.x: a strided scan per thread, then the wave
// butterfly and the four waves through LDS.
__global__ __launch_bounds__(256) void ga_best_kernel(const float* __restrict__ energies, int pop,
                                                      int32_t* __restrict__ best) {
    __shared__ float sk[4];
    __shared__ int si[4];
    const float* E = energies + (size_t)blockIdx.x * pop;
    float k = __builtin_inff();
    int i = 0x7fffffff;
    for (int m = (int)threadIdx.x; m < pop; m += 256) ga_min(k, i, ga_key(E[m]), m);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const float k2 = __shfl_xor(k, o);
        const int i2 = __shfl_xor(i, o);
        ga_min(k, i, k2, i2);
    }
    const int w = (int)threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sk[w] = k; si[w] = i; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < 4; ++v) ga_min(k, i, sk[v], si[v]);
        best[blockIdx.x] = i;
    }
}

// One thread per child gene: thread t writes gene t % G of child t / G. The
// child's parents are recomputed by each of its G threads from the same
// draws (a few cached loads), so no thread waits for another.
__global__ __launch_bounds__(256) void ga_child_kernel(docklaunch::GaParams p) {
    const int G = p.n_genes, P = p.pop;
    // the host keeps n_runs * pop * n_genes <= 2^31 - 1; the last block may
    // run past it, so the bound is checked before the index is narrowed
    const unsigned tu = blockIdx.x * 256u + threadIdx.x;
    if (tu >= (unsigned)(p.n_runs * P * G)) return;
    const int t = (int)tu;
    const int k = t / G, g = t - k * G;
    const int r = k / P, m = k - r * P;
    const float* gen = p.genotypes + (size_t)r * P * G;
    float v;
    if (p.elitism && m == 0) {
        v = gen[(size_t)p.best[r] * G + g];
    } else {
        const float* E = p.energies + (size_t)r * P;
        const int4 c = reinterpret_cast<const int4*>(p.cand)[k];
        const float* u = p.coins + (size_t)k * 3;
        auto pick = [&](int a, int b, float coin) {
            a = min(max(a, 0), P - 1);
            b = min(max(b, 0), P - 1);
            const bool a_fit = ga_key(E[a]) <= ga_key(E[b]);
            const int better = a_fit ? a : b, worse = a_fit ? b : a;
            return coin < p.p_tournament ? better : worse;
        };
        int src = pick(c.x, c.y, u[0]);
        if (u[2] < p.p_crossover) {
            const int2 cu = reinterpret_cast<const int2*>(p.cuts)[k];
            const int c0 = min(max(cu.x, 0), G), c1 = min(max(cu.y, 0), G);
            if (g >= min(c0, c1) && g < max(c0, c1)) src = pick(c.z, c.w, u[1]);
        }
        v = gen[(size_t)src * G + g];
        if (p.mut_coin[t] < p.p_mutation) v = __fadd_rn(v, p.mut_delta[t]);
    }
    p.children[t] = v;
}

// ---------------------------------------------------------------------------
// Local search on a share of the children (Sec. 2.1: the LGA improves the
// GA's genotypes by local search; AutoDock applies it at a rate below one):
// the rows whose draw is below the rate, in increasing order, then row
// gathers and scatters between the population and the compact search state.
// ---------------------------------------------------------------------------

// One block of 1024 threads: thread t owns rows [t * per, (t + 1) * per);
// per-thread counts, an exclusive scan over the block (wave scans, then the
// 16 wave totals), then each thread writes its selected rows in order.
__global__ __launch_bounds__(1024) void select_rows_kernel(const float* __restrict__ draws, int n, float rate,
                                                           int32_t* __restrict__ index,
                                                           int32_t* __restrict__ count) {
    __shared__ int wave_tot[16];
    const int t = (int)threadIdx.x;
    const int per = (int)(((long long)n + 1023) / 1024);
    const long long lo_l = (long long)t * per;
    const int lo = (int)(lo_l < n ? lo_l : n);
    const int hi = (int)(lo_l + per < n ? lo_l + per : n);
    int c = 0;
    for (int r = lo; r < hi; ++r) c += draws[r] < rate ? 1 : 0;
    // inclusive scan within the wave
    const int lane = t & 63, w = t >> 6;
    int incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wave_tot[w] = incl;
    __syncthreads();
    int before = 0;
    for (int v = 0; v < w; ++v) before += wave_tot[v];
    int pos = before + incl - c;
    for (int r = lo; r < hi; ++r)
        if (draws[r] < rate) index[pos++] = r;
    if (t == 1023) count[0] = before + incl;
}

// dst[k][c] = src[index[k]][c] (gather) or dst[index[k]][c] = src[k][c]
// (scatter), one thread per element; indices outside [0, n_rows) of the
// indexed side are skipped.
template <bool GATHER>
__global__ __launch_bounds__(256) void move_rows_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                        const int32_t* __restrict__ index, int m, int row,
                                                        int n_rows) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long long)m * row) return;
    const int k = (int)(e / row), c = (int)(e - (long long)k * row);
    const int r = index[k];
    if (r < 0 || r >= n_rows) return;
    if (GATHER)
        dst[e] = src[(size_t)r * row + c];
    else
        dst[(size_t)r * row + c] = src[e];
}

}  // namespace

namespace docklaunch {

hipError_t launch_select_rows(const float* draws, int n, float rate, int32_t* index, int32_t* count,
                              hipStream_t stream) {
    hipLaunchKernelGGL(select_rows_kernel, dim3(1), dim3(1024), 0, stream, draws, n, rate, index, count);
    return hipGetLastError();
}

hipError_t launch_move_rows(bool gather, const float* src, float* dst, const int32_t* index, int m, int row,
                            int n_rows, hipStream_t stream) {
    const long long total = (long long)m * row;
    if (total <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    if (gather)
        hipLaunchKernelGGL(move_rows_kernel<true>, dim3(blocks), dim3(256), 0, stream, src, dst, index, m, row, n_rows);
    else
        hipLaunchKernelGGL(move_rows_kernel<false>, dim3(blocks), dim3(256), 0, stream, src, dst, index, m, row, n_rows);
    return hipGetLastError();
}

hipError_t launch_ga_step(const GaParams& p, hipStream_t stream) {
    hipLaunchKernelGGL(ga_best_kernel, dim3((unsigned)p.n_runs), dim3(256), 0, stream, p.energies, p.pop, p.best);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long genes = (long long)p.n_runs * p.pop * p.n_genes;
    hipLaunchKernelGGL(ga_child_kernel, dim3((unsigned)((genes + 255) / 256)), dim3(256), 0, stream, p);
    return hipGetLastError();
}

}  // namespace docklaunch
