// sr_aux.hip -- helpers around the emission step: the prescribed standing-wave
// field on the Yee grid, the tile counting sort of the particles, the photon
// spectrum histogram, and error strings.
#include <math.h>

#include "sr_common.hpp"
#include "sr_hist.hpp"

namespace sr {
namespace {

// ------------------------------------------------------------ standing wave
// E = 2 a0 cos x (0, cos t, -sin t), B = 2 a0 sin x (0, -cos t, sin t), k = omega = 1.
// Each block owns 4*256 consecutive x cells and loops over rows (y, z); the x
// profile is computed once per thread in FP64 and rounded to binary32.
constexpr int kWaveXPerThread = 4;

__global__ __launch_bounds__(256) void standing_wave_kernel(float *ex, float *ey, float *ez,
                                                            float *bx, float *by, float *bz,
                                                            int nx, int64_t rows, int rows_per_block,
                                                            double dx, double a0, double t) {
    const int i0 = (blockIdx.x * 256 + threadIdx.x) * kWaveXPerThread;
    if (i0 >= nx) return;
    const double amp = 2.0 * a0, ct = cos(t), st = sin(t);
    float vey[kWaveXPerThread], vez[kWaveXPerThread], vby[kWaveXPerThread], vbz[kWaveXPerThread];
#pragma unroll
    for (int q = 0; q < kWaveXPerThread; ++q) {
        const int i = min(i0 + q, nx - 1);
        const double xe = (double)i * dx;          // Ey, Ez: no x offset
        const double xb = ((double)i + 0.5) * dx;  // By, Bz: x offset 1/2
        const double ce = cos(xe), sb = sin(xb);
        vey[q] = (float)(amp * ce * ct);
        vez[q] = (float)(-amp * ce * st);
        vby[q] = (float)(-amp * sb * ct);
        vbz[q] = (float)(amp * sb * st);
    }
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_block;
    const int64_t r1 = min(r0 + rows_per_block, rows);
    const bool vec = (nx % kWaveXPerThread) == 0;
    for (int64_t r = r0; r < r1; ++r) {
        const int64_t o = r * nx + i0;
        if (vec) {
            *(float4 *)(ex + o) = make_float4(0.f, 0.f, 0.f, 0.f);
            *(float4 *)(bx + o) = make_float4(0.f, 0.f, 0.f, 0.f);
            *(float4 *)(ey + o) = make_float4(vey[0], vey[1], vey[2], vey[3]);
            *(float4 *)(ez + o) = make_float4(vez[0], vez[1], vez[2], vez[3]);
            *(float4 *)(by + o) = make_float4(vby[0], vby[1], vby[2], vby[3]);
            *(float4 *)(bz + o) = make_float4(vbz[0], vbz[1], vbz[2], vbz[3]);
        } else {
            for (int q = 0; q < kWaveXPerThread && i0 + q < nx; ++q) {
                ex[o + q] = 0.f; bx[o + q] = 0.f;
                ey[o + q] = vey[q]; ez[o + q] = vez[q];
                by[o + q] = vby[q]; bz[o + q] = vbz[q];
            }
        }
    }
}

// ------------------------------------------------------------ tile sort
struct SortGeom {
    int dim;
    int n[3];
    int tile[3];
    int nt[3];          // tiles per axis
    float inv[3];
};

__device__ __forceinline__ uint32_t tile_key(const SortGeom &g, float x, float y, float z) {
    const float v[3] = {x, y, z};
    uint32_t key = 0, mul = 1;
    for (int a = 0; a < 3; ++a) {
        if (a >= g.dim) break;
        int c = (int)floorf(v[a] * g.inv[a]);
        c = min(max(c, 0), g.n[a] - 1);
        key += (uint32_t)(c / g.tile[a]) * mul;
        mul *= (uint32_t)g.nt[a];
    }
    return key;
}

__global__ void fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Runs of equal keys inside a wave (the input is nearly sorted after the first
// sort): the first lane of each run updates the counter once for the run.
struct WaveRun {
    bool head;
    int head_lane;   // first lane of this lane's run
    int len;         // run length (valid on the head lane)
};

__device__ __forceinline__ WaveRun wave_run(uint32_t k, bool valid) {
    const int lane = threadIdx.x & 63;
    const uint32_t kp = (uint32_t)__shfl_up((int)k, 1, 64);
    WaveRun r;
    r.head = valid && (lane == 0 || kp != k);
    const uint64_t hm = __ballot(r.head);
    const int nvalid = (int)__popcll(__ballot(valid));   // valid lanes form a prefix
    const uint64_t at_or_below = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const uint64_t below = hm & at_or_below;
    r.head_lane = below ? 63 - __clzll(below) : 0;
    const uint64_t above = hm & ~at_or_below;
    const int next = above ? __ffsll((long long)above) - 1 : 64;
    r.len = min(next, nvalid) - lane;
    return r;
}

// The block's smallest and largest key over the lanes that hold one (lane
// values kmin <= kmax, ignored where `any` is false); false when no lane holds
// one.  Keys are below 2^31 (the tile count is checked on the host).
__device__ __forceinline__ bool block_key_range(uint32_t kmin, uint32_t kmax, bool any,
                                                uint32_t &lo, uint32_t &hi) {
    __shared__ int rlo[4], rhi[4];
    int a = any ? (int)kmin : 0x7fffffff, b = any ? (int)kmax : -1;
    for (int o = 32; o > 0; o >>= 1) {
        a = min(a, __shfl_xor(a, o, 64));
        b = max(b, __shfl_xor(b, o, 64));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { rlo[wave] = a; rhi[wave] = b; }
    __syncthreads();
    a = rlo[0];
    b = rhi[0];
    for (int w = 1; w < 4; ++w) { a = min(a, rlo[w]); b = max(b, rhi[w]); }
    lo = (uint32_t)a;
    hi = (uint32_t)b;
    return b >= a;
}

// A block takes kSortPer consecutive particles, kSortPPT per thread in rounds
// of 256 (coalesced loads, all in flight together), and groups their keys in
// LDS: particles sorted some steps ago fall in a few nearby tiles, so one
// global atomic per distinct key of the block replaces one per run of equal
// keys in each wave.  Keys within a span of kSortSpan index an LDS array
// directly; a block whose keys span more (particles that drifted across tile
// rows and planes) groups them in an LDS hash table of kHashSlots slots, twice
// the most distinct keys a block can hold.
constexpr int kSortPPT = 2;
constexpr int kSortPer = 256 * kSortPPT;
constexpr uint32_t kSortSpan = 4096;
constexpr uint32_t kHashSlots = 1024;
constexpr uint32_t kHashEmpty = 0xFFFFFFFFu;
static_assert(kHashSlots >= 2 * kSortPer && 2 * kHashSlots <= kSortSpan, "LDS table sizes");

// The slot of key k in the block's table (inserting it if absent); linear
// probing from a multiplicative hash.
__device__ __forceinline__ uint32_t hash_slot(uint32_t *hk, uint32_t k) {
    uint32_t h = (k * 2654435761u) >> 22;   // 10 bits
    for (;;) {
        const uint32_t prev = atomicCAS(&hk[h], kHashEmpty, k);
        if (prev == kHashEmpty || prev == k) return h;
        h = (h + 1u) & (kHashSlots - 1u);
    }
}
// The slot of a key already in the table.
__device__ __forceinline__ uint32_t hash_find(const uint32_t *hk, uint32_t k) {
    uint32_t h = (k * 2654435761u) >> 22;
    while (hk[h] != k) h = (h + 1u) & (kHashSlots - 1u);
    return h;
}

// First particle of the block: neighbouring particle ranges on one XCD, so
// their tiles' counters and segments stay in that XCD's L2.
__device__ __forceinline__ int64_t sort_block_first() {
    return xcd_chunk(blockIdx.x, gridDim.x) * kSortPer + threadIdx.x;
}

// Lane range of the thread's valid keys.
__device__ __forceinline__ bool lane_key_range(const uint32_t (&k)[kSortPPT],
                                               const bool (&valid)[kSortPPT], uint32_t &a,
                                               uint32_t &b) {
    a = 0xFFFFFFFFu;
    b = 0u;
#pragma unroll
    for (int r = 0; r < kSortPPT; ++r)
        if (valid[r]) {
            a = min(a, k[r]);
            b = max(b, k[r]);
        }
    return valid[0];   // valid particles form a prefix of the rounds
}

__global__ __launch_bounds__(256) void sort_count(const float *x, const float *y, const float *z,
                                                  int64_t n, SortGeom g, uint32_t *counts) {
    __shared__ uint32_t lc[kSortSpan];
    const int64_t i0 = sort_block_first();
    uint32_t k[kSortPPT];
    bool valid[kSortPPT];
    float px[kSortPPT], py[kSortPPT], pz[kSortPPT];
#pragma unroll
    for (int r = 0; r < kSortPPT; ++r) {
        const int64_t i = i0 + r * 256;
        valid[r] = i < n;
        px[r] = valid[r] ? x[i] : 0.0f;
        py[r] = valid[r] ? y[i] : 0.0f;
        pz[r] = valid[r] && g.dim == 3 ? z[i] : 0.0f;
    }
#pragma unroll
    for (int r = 0; r < kSortPPT; ++r) k[r] = valid[r] ? tile_key(g, px[r], py[r], pz[r]) : 0xFFFFFFFFu;
    uint32_t a, b, lo, hi;
    const bool any = lane_key_range(k, valid, a, b);
    if (!block_key_range(a, b, any, lo, hi)) return;   // no valid lane (block-wide)
    WaveRun run[kSortPPT];
#pragma unroll
    for (int r = 0; r < kSortPPT; ++r) run[r] = wave_run(k[r], valid[r]);
    if (hi - lo < kSortSpan) {
        for (uint32_t e = threadIdx.x; e <= hi - lo; e += blockDim.x) lc[e] = 0u;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortPPT; ++r)
            if (valid[r] && run[r].head) atomicAdd(&lc[k[r] - lo], (uint32_t)run[r].len);
        __syncthreads();
        for (uint32_t e = threadIdx.x; e <= hi - lo; e += blockDim.x)
            if (lc[e]) atomicAdd(&counts[lo + e], lc[e]);
    } else {
        uint32_t *hk = lc, *hc = lc + kHashSlots;
        for (uint32_t e = threadIdx.x; e < kHashSlots; e += blockDim.x) {
            hk[e] = kHashEmpty;
            hc[e] = 0u;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortPPT; ++r)
            if (valid[r] && run[r].head) atomicAdd(&hc[hash_slot(hk, k[r])], (uint32_t)run[r].len);
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < kHashSlots; e += blockDim.x)
            if (hc[e]) atomicAdd(&counts[hk[e]], hc[e]);
    }
}

// exclusive scan in blocks of 1024 (256 threads x 4)
__global__ __launch_bounds__(256) void scan_blocks(const uint32_t *in, uint32_t *out, int64_t n,
                                                   uint32_t *block_sums) {
    __shared__ uint32_t s[256];
    const int64_t b0 = (int64_t)blockIdx.x * 1024;
    uint32_t v[4], sum = 0;
    for (int q = 0; q < 4; ++q) {
        const int64_t i = b0 + threadIdx.x * 4 + q;
        v[q] = i < n ? in[i] : 0u;
        sum += v[q];
    }
    s[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t add = threadIdx.x >= o ? s[threadIdx.x - o] : 0u;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = s[threadIdx.x] - sum;
    for (int q = 0; q < 4; ++q) {
        const int64_t i = b0 + threadIdx.x * 4 + q;
        if (i < n) out[i] = run;
        run += v[q];
    }
    if (threadIdx.x == 255 && block_sums) block_sums[blockIdx.x] = s[255];
}

__global__ void scan_add(uint32_t *out, int64_t n, const uint32_t *block_prefix) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += block_prefix[i / 1024];
}

// Each particle goes to its slot among the tile's particles, counted from the
// tile's offset: offsets[key] serves as the tile's cursor (it ends as the
// tile's end).  The key is computed again from the position, by the same
// function on the same values as in sort_count, so it needs no buffer.  Slots
// are handed out per block and key (LDS), then per block from the cursor: one
// global atomic per distinct key of the block.
__global__ __launch_bounds__(256) void sort_scatter(sr_particles_f32 src, sr_particles_f32 dst,
                                                    SortGeom g, uint32_t *cursor) {
    __shared__ uint32_t lc[kSortSpan];
    const int64_t i0 = sort_block_first();
    // the particles' values are read first: they do not depend on where they go
    float v[kSortPPT][7];
    uint32_t id[kSortPPT], k[kSortPPT];
    bool valid[kSortPPT];
#pragma unroll
    for (int r = 0; r < kSortPPT; ++r) {
        const int64_t i = i0 + r * 256;
        valid[r] = i < src.n;
#pragma unroll
        for (int c = 0; c < 7; ++c) v[r][c] = 0.0f;
        id[r] = 0u;
        k[r] = 0xFFFFFFFFu;
        if (valid[r]) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (src.x[a]) v[r][a] = src.x[a][i];
                v[r][3 + a] = src.p[a][i];
            }
            v[r][6] = src.w[i];
            id[r] = src.id[i];
        }
    }
#pragma unroll
    for (int r = 0; r < kSortPPT; ++r)
        if (valid[r]) k[r] = tile_key(g, v[r][0], v[r][1], v[r][2]);
    uint32_t a, b, lo, hi;
    const bool any = lane_key_range(k, valid, a, b);
    if (!block_key_range(a, b, any, lo, hi)) return;   // no valid lane (block-wide)
    WaveRun run[kSortPPT];
    uint32_t base[kSortPPT];
#pragma unroll
    for (int r = 0; r < kSortPPT; ++r) {
        run[r] = wave_run(k[r], valid[r]);
        base[r] = 0u;
    }
    const bool local = hi - lo < kSortSpan;
    uint32_t *hk = lc, *hc = lc + kHashSlots;
    if (local) {
        for (uint32_t e = threadIdx.x; e <= hi - lo; e += blockDim.x) lc[e] = 0u;
        __syncthreads();
        // each run's place among the block's particles of its tile
#pragma unroll
        for (int r = 0; r < kSortPPT; ++r)
            if (valid[r] && run[r].head) base[r] = atomicAdd(&lc[k[r] - lo], (uint32_t)run[r].len);
        __syncthreads();
        // the block's first slot in the tile
        for (uint32_t e = threadIdx.x; e <= hi - lo; e += blockDim.x) {
            const uint32_t c = lc[e];
            if (c) lc[e] = atomicAdd(&cursor[lo + e], c);
        }
        __syncthreads();
    } else {
        for (uint32_t e = threadIdx.x; e < kHashSlots; e += blockDim.x) {
            hk[e] = kHashEmpty;
            hc[e] = 0u;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortPPT; ++r)
            if (valid[r] && run[r].head)
                base[r] = atomicAdd(&hc[hash_slot(hk, k[r])], (uint32_t)run[r].len);
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < kHashSlots; e += blockDim.x) {
            const uint32_t c = hc[e];
            if (c) hc[e] = atomicAdd(&cursor[hk[e]], c);
        }
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < kSortPPT; ++r) {
        const uint32_t rb = (uint32_t)__shfl((int)base[r], run[r].head_lane, 64);
        if (!valid[r]) continue;
        const uint32_t slot0 = local ? lc[k[r] - lo] : hc[hash_find(hk, k[r])];
        const int64_t j = (int64_t)slot0 + rb + (lane - run[r].head_lane);
        if (j >= src.n) continue;   // unreachable: both kernels compute the same key
#pragma unroll
        for (int a2 = 0; a2 < 3; ++a2) {
            if (src.x[a2] && dst.x[a2]) dst.x[a2][j] = v[r][a2];
            dst.p[a2][j] = v[r][3 + a2];
        }
        dst.w[j] = v[r][6];
        dst.id[j] = id[r];
    }
}

// ------------------------------------------------------------ histogram
// The block work lives in sr_hist.hpp (the step epilogue uses it too).
__global__ __launch_bounds__(256) void hist_kernel(sr_photon_buf ph, const int64_t *start,
                                                   int64_t n_chunks, int64_t n, float l2lo,
                                                   float scale, int nbins, double *work) {
    extern __shared__ double sh[];   // [2*nbins]
    hist_block(ph, start, n_chunks, n, l2lo, scale, nbins, work, blockIdx.x, gridDim.x, sh);
}

__global__ __launch_bounds__(256) void hist_reduce(const double *work, int nblocks, int nvals,
                                                   double *hist) {
    hist_reduce_value(work, nblocks, nvals, hist, blockIdx.x);
}

// Energy-weighted angular map of the stored photons (the angular distribution
// of emitted energy of section "Comparison and benchmarking", Fig. 4): theta is
// the angle from the axis, binned uniformly on [0, pi/2) (the front
// hemisphere); phi is the azimuth about the axis from e1 towards e2, binned on
// [0, 2 pi).  Photons with dir . axis <= 0 go to the last bin (the back
// hemisphere).  One lane per chunk, as hist_kernel; block partials to work.
constexpr int kMaxAngularBins = 4096;
__global__ __launch_bounds__(256) void angular_kernel(sr_photon_buf ph, const int64_t *start,
                                                      int64_t n_chunks, int64_t n, float3 ax,
                                                      float3 e1, float3 e2, int n_theta,
                                                      int n_phi, double *work) {
    extern __shared__ double sh[];   // [n_theta * n_phi + 1]
    const int nvals = n_theta * n_phi + 1;
    for (int b = threadIdx.x; b < nvals; b += blockDim.x) sh[b] = 0.0;
    __syncthreads();
    const float t_scale = (float)n_theta * 0.63661977236758134f;   // n_theta / (pi/2)
    const float p_scale = (float)n_phi * 0.15915494309189535f;     // n_phi / (2 pi)
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_chunks;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s0 = start ? start[c] : c * (int64_t)kChunk;
        const int64_t e0 = start ? start[c + 1] : min(s0 + (int64_t)kChunk, n);
        const int64_t cap = (e0 - s0) * ph.per_particle;
        const int64_t cnt = min((int64_t)ph.seg_count[c], cap);
        const int64_t base = s0 * ph.per_particle;
        for (int64_t q = 0; q < cnt; ++q) {
            const int64_t o = base + q;
            const float e = ph.eps[o] * ph.w[o];
            const float d0 = ph.dir[0][o], d1 = ph.dir[1][o], d2 = ph.dir[2][o];
            const float cz = d0 * ax.x + d1 * ax.y + d2 * ax.z;
            int bin = nvals - 1;
            if (cz > 0.0f) {
                const float theta = acosf(fminf(cz, 1.0f));
                const int it = min((int)(theta * t_scale), n_theta - 1);
                float phi = atan2f(d0 * e2.x + d1 * e2.y + d2 * e2.z, d0 * e1.x + d1 * e1.y + d2 * e1.z);
                if (phi < 0.0f) phi += 6.2831853071795865f;
                const int ip = min(max((int)(phi * p_scale), 0), n_phi - 1);
                bin = it * n_phi + ip;
            }
            atomicAdd(&sh[bin], (double)e);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nvals; b += blockDim.x)
        work[(int64_t)blockIdx.x * nvals + b] = sh[b];
}

}  // namespace
}  // namespace sr

using namespace sr;

extern "C" int64_t sr_angular_work(int32_t n_theta, int32_t n_phi) {
    if (n_theta < 1 || n_phi < 1 || (int64_t)n_theta * n_phi > kMaxAngularBins) return -1;
    return (int64_t)kHistBlocks * ((int64_t)n_theta * n_phi + 1);
}

extern "C" int sr_angular_histogram(const sr_photon_buf *ph, const sr_chunking *chunks, int64_t n,
                                    const double axis[3], const double ref[3], int32_t n_theta,
                                    int32_t n_phi, double *hist, double *work, void *stream) {
    if (!ph || !chunks || !axis || !ref || !hist || !work || n < 0 || n_theta < 1 || n_phi < 1 ||
        (int64_t)n_theta * n_phi > kMaxAngularBins || !ph->seg_count)
        return SR_E_INVAL;
    const double an = sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
    if (!(an > 0.0)) return SR_E_INVAL;
    const double a[3] = {axis[0] / an, axis[1] / an, axis[2] / an};
    const double ra = ref[0] * a[0] + ref[1] * a[1] + ref[2] * a[2];
    double u[3] = {ref[0] - ra * a[0], ref[1] - ra * a[1], ref[2] - ra * a[2]};
    const double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (!(un > 1e-12 * sqrt(ref[0] * ref[0] + ref[1] * ref[1] + ref[2] * ref[2])) || !(un > 0.0))
        return SR_E_INVAL;   // ref must not be parallel to the axis
    for (int q = 0; q < 3; ++q) u[q] /= un;
    const double v[3] = {a[1] * u[2] - a[2] * u[1], a[2] * u[0] - a[0] * u[2],
                         a[0] * u[1] - a[1] * u[0]};
    const int64_t n_chunks = chunks->start ? chunks->n_chunks : (n + kChunk - 1) / kChunk;
    if (n_chunks == 0 || ph->per_particle == 0) return SR_OK;
    if (!ph->eps || !ph->w || !ph->dir[0] || !ph->dir[1] || !ph->dir[2]) return SR_E_INVAL;
    const int nvals = n_theta * n_phi + 1;
    const int64_t groups = (n_chunks + 255) / 256;   // one lane per chunk
    const int nb = (int)(groups < kHistBlocks ? groups : kHistBlocks);
    hipStream_t st = (hipStream_t)stream;
    angular_kernel<<<nb, 256, sizeof(double) * nvals, st>>>(
        *ph, chunks->start, n_chunks, n, make_float3((float)a[0], (float)a[1], (float)a[2]),
        make_float3((float)u[0], (float)u[1], (float)u[2]),
        make_float3((float)v[0], (float)v[1], (float)v[2]), n_theta, n_phi, work);
    hist_reduce<<<nvals, 256, 0, st>>>(work, nb, nvals, hist);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

extern "C" int sr_field_standing_wave(float *e[3], float *b[3], const sr_grid *grid, double a0,
                                      double t, void *stream) {
    if (!e || !b || !grid) return SR_E_INVAL;
    for (int q = 0; q < 3; ++q)
        if (!e[q] || !b[q]) return SR_E_INVAL;
    if (grid->dim != 2 && grid->dim != 3) return SR_E_INVAL;
    const int64_t nx = grid->n[0], ny = grid->n[1], nz = grid->dim == 3 ? grid->n[2] : 1;
    if (nx < 1 || ny < 1 || nz < 1 || nx > (1 << 24) || !(grid->dx[0] > 0.0)) return SR_E_INVAL;
    const int64_t rows = ny * nz;
    const unsigned bx = (unsigned)((nx + 256 * kWaveXPerThread - 1) / (256 * kWaveXPerThread));
    // about 256 blocks (one per CU), each writing a band of rows with its x
    // profile reused: fewer blocks recompute the FP64 profile less often
    int64_t by = (256 + bx - 1) / bx;
    if (by > rows) by = rows;
    if (by > 65535) by = 65535;
    const int rows_per_block = (int)((rows + by - 1) / by);
    by = (rows + rows_per_block - 1) / rows_per_block;
    standing_wave_kernel<<<dim3(bx, (unsigned)by), 256, 0, (hipStream_t)stream>>>(
        e[0], e[1], e[2], b[0], b[1], b[2], (int)nx, rows, rows_per_block, grid->dx[0], a0, t);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

static bool sort_geom(const sr_grid *grid, const int32_t tile[3], SortGeom &g, int64_t &n_tiles) {
    if (!grid || !tile || (grid->dim != 2 && grid->dim != 3)) return false;
    g.dim = grid->dim;
    n_tiles = 1;
    for (int a = 0; a < 3; ++a) {
        if (a >= g.dim) {
            g.n[a] = 1; g.tile[a] = 1; g.nt[a] = 1; g.inv[a] = 0.0f;
            continue;
        }
        if (grid->n[a] < 1 || grid->n[a] > (1 << 24) || tile[a] < 1 || !(grid->dx[a] > 0.0))
            return false;
        g.n[a] = (int)grid->n[a];
        g.tile[a] = tile[a];
        g.nt[a] = (int)((grid->n[a] + tile[a] - 1) / tile[a]);
        g.inv[a] = (float)(1.0 / grid->dx[a]);
        n_tiles *= g.nt[a];
    }
    return n_tiles > 0 && n_tiles < ((int64_t)1 << 31);
}

extern "C" int64_t sr_sort_work(const sr_grid *grid, const int32_t tile[3], int64_t n) {
    SortGeom g;
    int64_t nt;
    if (n < 0 || !sort_geom(grid, tile, g, nt)) return -1;
    const int64_t nblk = (nt + 1023) / 1024;
    // counts, offsets, one spare (n_tiles each), block sums + their prefix
    return (int64_t)sizeof(uint32_t) * (3 * nt + 2 * (nblk + 1024));
}

extern "C" int sr_sort_particles(const sr_particles_f32 *src, sr_particles_f32 *dst,
                                 const sr_grid *grid, const int32_t tile[3], void *work,
                                 void *stream) {
    SortGeom g;
    int64_t nt;
    if (!src || !dst || !work || !sort_geom(grid, tile, g, nt)) return SR_E_INVAL;
    const int64_t n = src->n;
    if (n < 0 || dst->n != n || n > 0xFFFFFFFFll) return SR_E_INVAL;
    if (n == 0) return SR_OK;
    for (int a = 0; a < 3; ++a)
        if (!src->p[a] || !dst->p[a]) return SR_E_INVAL;
    if (!src->x[0] || !src->x[1] || (g.dim == 3 && !src->x[2]) || !src->w || !src->id ||
        !dst->x[0] || !dst->x[1] || (g.dim == 3 && !dst->x[2]) || !dst->w || !dst->id)
        return SR_E_INVAL;
    const int64_t nblk = (nt + 1023) / 1024;
    if (nblk > 1024 * 1024) return SR_E_UNSUPPORTED;
    uint32_t *counts = (uint32_t *)work;
    uint32_t *offsets = counts + nt;
    uint32_t *bsum = offsets + 2 * nt;   // after the spare n_tiles words
    uint32_t *bpre = bsum + nblk + 1024;
    hipStream_t st = (hipStream_t)stream;
    const unsigned g256 = (unsigned)((nt + 255) / 256);
    fill_u32<<<g256, 256, 0, st>>>(counts, nt, 0u);
    const unsigned gsort = (unsigned)((n + kSortPer - 1) / kSortPer);
    sort_count<<<gsort, 256, 0, st>>>(src->x[0], src->x[1], src->x[2], n, g, counts);
    scan_blocks<<<(unsigned)nblk, 256, 0, st>>>(counts, offsets, nt, bsum);
    if (nblk > 1) {
        // scan of the block sums: at most 1024*1024 tiles, so one more level of
        // blocks and a final single-block scan suffice
        const int64_t nblk2 = (nblk + 1023) / 1024;
        uint32_t *b2sum = bpre + nblk;   // fits: bpre has nblk + 1024 slots
        scan_blocks<<<(unsigned)nblk2, 256, 0, st>>>(bsum, bpre, nblk, nblk2 > 1 ? b2sum : nullptr);
        if (nblk2 > 1) {
            uint32_t *b2pre = bsum + nblk;   // bsum has nblk + 1024 slots
            scan_blocks<<<1, 256, 0, st>>>(b2sum, b2pre, nblk2, nullptr);
            scan_add<<<(unsigned)((nblk + 255) / 256), 256, 0, st>>>(bpre, nblk, b2pre);
        }
        scan_add<<<(unsigned)((nt + 255) / 256), 256, 0, st>>>(offsets, nt, bpre);
    }
    sort_scatter<<<gsort, 256, 0, st>>>(*src, *dst, g, offsets);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

extern "C" int64_t sr_hist_work(int32_t n_bins) {
    if (n_bins < 1 || n_bins > kMaxBins) return -1;
    return (int64_t)kHistBlocks * 2 * n_bins;
}

extern "C" int sr_spectrum_histogram(const sr_photon_buf *ph, const sr_chunking *chunks,
                                     int64_t n, double eps_lo, double eps_hi, int32_t n_bins,
                                     double *hist, double *work, void *stream) {
    if (!ph || !chunks || !hist || !work || n < 0 || n_bins < 1 || n_bins > kMaxBins ||
        !(eps_lo > 0.0) || !(eps_hi > eps_lo) || !ph->seg_count)
        return SR_E_INVAL;
    const int64_t n_chunks = chunks->start ? chunks->n_chunks : (n + kChunk - 1) / kChunk;
    if (n_chunks == 0 || ph->per_particle == 0) return SR_OK;
    if (!ph->eps || !ph->w) return SR_E_INVAL;
    const float l2lo = (float)log2(eps_lo);
    const float scale = (float)(n_bins / (log2(eps_hi) - log2(eps_lo)));
    const int nb = hist_blocks(n_chunks);
    hipStream_t st = (hipStream_t)stream;
    hist_kernel<<<nb, 256, sizeof(double) * 2 * n_bins, st>>>(*ph, chunks->start, n_chunks, n,
                                                               l2lo, scale, n_bins, work);
    hist_reduce<<<2 * n_bins, 256, 0, st>>>(work, nb, 2 * n_bins, hist);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

extern "C" const char *sr_strerror(int code) {
    switch (code) {
        case SR_OK: return "ok";
        case SR_E_INVAL: return "invalid argument";
        case SR_E_HIP: return "HIP runtime error";
        case SR_E_NOMEM: return "device allocation failed";
        case SR_E_UNSUPPORTED: return "unsupported request";
        default: return "unknown error code";
    }
}
