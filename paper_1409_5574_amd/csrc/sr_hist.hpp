// sr_hist.hpp -- the block-level work of the photon energy spectrum (section
// "Comparison and benchmarking": the energy-weighted spectrum of the emitted
// photons), shared by the histogram entry point and the step epilogue.
#pragma once

#include "sr_common.hpp"

namespace sr {

constexpr int kHistBlocks = 1024;  // most blocks of the accumulation pass
constexpr int kMaxBins = 1024;
constexpr int kHistChunks = 64;    // chunks per block and group (four lanes each)

// Four lanes per chunk: the lanes of a chunk walk its stored photons in turn
// and add w eps and w to bins of log2 eps in the block's LDS histogram
// sh[2 nbins] (FP64 LDS atomics, which cost about one lane per few cycles, so
// the photons are spread over many blocks).  Block hb of nblocks strides over
// groups of kHistChunks chunks and writes its histogram to work[hb].  Call
// with the whole block of 256 threads.
__device__ __forceinline__ void hist_block(const sr_photon_buf &ph, const int64_t *start,
                                           int64_t n_chunks, int64_t n, float l2lo, float scale,
                                           int nbins, double *work, int hb, int nblocks,
                                           double *sh) {
    for (int b = threadIdx.x; b < 2 * nbins; b += blockDim.x) sh[b] = 0.0;
    __syncthreads();
    const int sub = threadIdx.x & 3;
    for (int64_t c = (int64_t)hb * kHistChunks + (threadIdx.x >> 2); c < n_chunks;
         c += (int64_t)nblocks * kHistChunks) {
        const int64_t s0 = start ? start[c] : c * (int64_t)kChunk;
        const int64_t e0 = start ? start[c + 1] : min(s0 + (int64_t)kChunk, n);
        const int64_t cap = (e0 - s0) * ph.per_particle;
        const int64_t cnt = min((int64_t)ph.seg_count[c], cap);
        const int64_t base = s0 * ph.per_particle;
        // photons sub, sub + 4, ...: two of the lane's at a time, loads in flight
        for (int64_t q0 = sub; q0 < cnt; q0 += 8) {
            float eps[2], w[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                eps[j] = 0.0f;
                w[j] = 0.0f;
                if (q0 + 4 * j < cnt) {
                    eps[j] = ph.eps[base + q0 + 4 * j];
                    w[j] = ph.w[base + q0 + 4 * j];
                }
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (!(eps[j] > 0.0f)) continue;
                const float u = (__log2f(eps[j]) - l2lo) * scale;
                if (u < 0.0f || u >= (float)nbins) continue;
                const int bin = (int)u;
                atomicAdd(&sh[bin], (double)w[j] * (double)eps[j]);
                atomicAdd(&sh[nbins + bin], (double)w[j]);
            }
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < 2 * nbins; b += blockDim.x)
        work[(int64_t)hb * 2 * nbins + b] = sh[b];
}

// hist[b] += the sum over blocks of work[block][b], in a fixed order (a block
// of 256 threads per value b).
__device__ __forceinline__ void hist_reduce_value(const double *work, int nblocks, int nvals,
                                                  double *hist, int b) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += 256) acc += work[(int64_t)k * nvals + b];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) hist[b] += s[0];
}

// Blocks of the accumulation pass for n_chunks chunks.
inline int hist_blocks(int64_t n_chunks) {
    const int64_t groups = (n_chunks + kHistChunks - 1) / kHistChunks;
    return (int)(groups < kHistBlocks ? groups : kHistBlocks);
}

}  // namespace sr
