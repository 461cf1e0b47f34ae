// sr_step.hip -- the per-particle, per-step emission kernel and its ledger
// reduction.
//
// One thread per macro-electron, one block (256 threads, 4 waves) per chunk of
// the particle array.  Per particle (section "Numerical implementation" and
// the recipe at the end of section "Monte Carlo method"):
//   gather E, B at x^n -> Boris push -> H_eff (eq:effective_H, dp_perp/p <= 1)
//   -> omega_c = 1.5 H gamma^2, chi = hbar_n H gamma -> K trials
//   -> photon append -> recoil -> position push.
// Photon append uses no global atomics: each chunk owns a segment of the
// photon buffer, the wave ballot + lane prefix (mbcnt) give every emitted
// trial its slot inside the wave, and the four wave totals are combined in
// LDS.  The FP64 ledger is reduced per block and written as one partial row per
// chunk, then summed in a fixed order by ledger_reduce (deterministic).  The
// step epilogue runs that reduction and the photon spectrum histogram together
// in two launches.
#include <math.h>
#include <stddef.h>

#include <mutex>
#include <type_traits>

#include <hip/hip_ext.h>

#include "sr_hist.hpp"
#include "sr_mlp.hpp"

namespace sr {
namespace {

// Outputs written once per wave (photon records, segment counts, ledger
// partials, status).  The kernel reads these pointers through cold_args() at
// the point of use so they do not occupy scalar registers for the whole kernel.
struct PhotonOut {
    float *eps, *w, *dir[3], *pos[3];
    uint32_t *parent, *step;
    uint8_t *k;
    uint32_t *seg_count;
    double *partials;
};

template <typename R>
struct StepArgs {
    int64_t n;
    R *x[3];
    R *p[3];
    const R *w;
    const uint32_t *id;
    const float *f[6];
    GridK g;
    R dt, inv_dt;
    uint32_t seed_lo, seed_hi, step;
    int K, recoil, dn_policy, kin_cut, push_position, has_pos;
    R hbar_n;
    float rate_c;      // dt sqrt3/(2 pi) alpha        (x H gives the trial rate)
    float direct_c;    // dt 5/(2 sqrt3) alpha          (x H r gives the direct rate)
    float e_grid;      // hbar_n omega_grid: no photon below this energy (0: no floor)
    R ll_c;            // (2/3)(alpha/hbar_n) dt        (x chi^2 beta^2 gives the LL loss)
    TableDev tab;
    const __bf16 *mlp;              // network parameters (MLP sampler)
    const uint8_t *mlp_fallback;    // per-chi-bin fallback map (MLP sampler)
    const int64_t *start;
    int64_t n_chunks;
    int64_t per_particle;
    PhotonOut ph;
};

template <typename R>
__device__ __forceinline__ void setup_axis(const GridK &g, int ax, R x, Axis<R> &A);
template <>
__device__ __forceinline__ void setup_axis<float>(const GridK &g, int ax, float x, Axis<float> &A) {
    axis_setup(x, g.inv_hi[ax], g.inv_lo[ax], g.n[ax], A);
}
template <>
__device__ __forceinline__ void setup_axis<double>(const GridK &g, int ax, double x,
                                                   Axis<double> &A) {
    axis_setup(x, g.inv_d[ax], g.n[ax], A);
}

template <typename R, int DIM>
__device__ __forceinline__ void gather_grid(const StepArgs<R> &a, const R pos[3], R E[3], R B[3]) {
    Axis<R> X, Y, Z;
    setup_axis<R>(a.g, 0, pos[0], X);
    setup_axis<R>(a.g, 1, pos[1], Y);
    if (DIM == 3) setup_axis<R>(a.g, 2, pos[2], Z);
    else Z = Y;
    const int nx = a.g.n[0], ny = a.g.n[1];
    const XPair P0 = x_pair(X.i0, nx), P1 = x_pair(X.i1, nx);
    // Yee offsets: Ex(1/2,0,0) Ey(0,1/2,0) Ez(0,0,1/2) Bx(0,1/2,1/2) By(1/2,0,1/2) Bz(1/2,1/2,0)
    E[0] = cic<R, DIM>(a.f[0], X, Y, Z, P0, P1, true, false, false, nx, ny);
    E[1] = cic<R, DIM>(a.f[1], X, Y, Z, P0, P1, false, true, false, nx, ny);
    E[2] = cic<R, DIM>(a.f[2], X, Y, Z, P0, P1, false, false, true, nx, ny);
    B[0] = cic<R, DIM>(a.f[3], X, Y, Z, P0, P1, false, true, true, nx, ny);
    B[1] = cic<R, DIM>(a.f[4], X, Y, Z, P0, P1, true, false, true, nx, ny);
    B[2] = cic<R, DIM>(a.f[5], X, Y, Z, P0, P1, true, true, false, nx, ny);
}

template <typename R> __device__ __forceinline__ R box_len(const GridK &g, int q);
template <> __device__ __forceinline__ float box_len<float>(const GridK &g, int q) { return g.L[q]; }
template <> __device__ __forceinline__ double box_len<double>(const GridK &g, int q) { return g.Ld[q]; }
template <typename R> __device__ __forceinline__ R uniform_e(const GridK &g, int q);
template <typename R> __device__ __forceinline__ R uniform_b(const GridK &g, int q);
template <> __device__ __forceinline__ float uniform_e<float>(const GridK &g, int q) { return g.e0[q]; }
template <> __device__ __forceinline__ double uniform_e<double>(const GridK &g, int q) { return g.e0d[q]; }
template <> __device__ __forceinline__ float uniform_b<float>(const GridK &g, int q) { return g.b0[q]; }
template <> __device__ __forceinline__ double uniform_b<double>(const GridK &g, int q) { return g.b0d[q]; }

// Gather, Boris push and H_eff of one particle (section "Numerical
// implementation"; eq:effective_H with the limiter dp_perp/p <= 1), shared by
// the emission step and the evaluation entry point.
template <typename R>
struct Pushed {
    R pn[3];      // p^{n+1/2}
    R pb[3];      // mean momentum of the step
    R p2;         // |pb|^2
    R gb;         // mean gamma of the step
    R g_new;      // gamma(p^{n+1/2})
    R pbm;        // |pb|
    R H;          // H_eff
    R chi;        // hbar_n H_eff gamma_bar
    bool bad;     // the push is not finite (a non-finite field value or momentum)
};

template <typename R>
__device__ __forceinline__ Pushed<R> push_fields(const StepArgs<R> &a, const R p0[3], const R E[3],
                                                 const R B[3]);

template <typename R, int DIM>
__device__ __forceinline__ Pushed<R> push_heff(const StepArgs<R> &a, const R pos[3],
                                               const R p0[3]) {
    R E[3], B[3];
    if (DIM == 0) {
        for (int q = 0; q < 3; ++q) { E[q] = uniform_e<R>(a.g, q); B[q] = uniform_b<R>(a.g, q); }
    } else {
        gather_grid<R, DIM>(a, pos, E, B);
    }
    return push_fields<R>(a, p0, E, B);
}

// The same, with the fields interpolated from the block's LDS field box (3D).
template <typename R>
__device__ __forceinline__ Pushed<R> push_box(const StepArgs<R> &a, const R pos[3], const R p0[3],
                                              const float (*box)[kBoxCells], const FieldBox &fb) {
    Axis<R> X, Y, Z;
    setup_axis<R>(a.g, 0, pos[0], X);
    setup_axis<R>(a.g, 1, pos[1], Y);
    setup_axis<R>(a.g, 2, pos[2], Z);
    const int n[3] = {a.g.n[0], a.g.n[1], a.g.n[2]};
    // Yee offsets as in gather_grid
    const R E[3] = {cic_box<R>(box[0], X, Y, Z, fb, n, true, false, false),
                    cic_box<R>(box[1], X, Y, Z, fb, n, false, true, false),
                    cic_box<R>(box[2], X, Y, Z, fb, n, false, false, true)};
    const R B[3] = {cic_box<R>(box[3], X, Y, Z, fb, n, false, true, true),
                    cic_box<R>(box[4], X, Y, Z, fb, n, true, false, true),
                    cic_box<R>(box[5], X, Y, Z, fb, n, true, true, false)};
    return push_fields<R>(a, p0, E, B);
}

template <typename R>
__device__ __forceinline__ Pushed<R> push_fields(const StepArgs<R> &a, const R p0[3], const R E[3],
                                                 const R B[3]) {
    Pushed<R> o;
    // ---- Boris push (q = -1), keeping the momentum increment d explicitly
    const R h = (R)(-0.5) * a.dt;
    const R um[3] = {p0[0] + h * E[0], p0[1] + h * E[1], p0[2] + h * E[2]};
    const R gm = sqrt_r<R>((R)1 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    const R hg = h * rcp_r<R>(gm);
    const R t[3] = {hg * B[0], hg * B[1], hg * B[2]};
    const R t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    const R sc = (R)2 * rcp_r<R>((R)1 + t2);
    const R sv[3] = {sc * t[0], sc * t[1], sc * t[2]};
    const R up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]),
                     um[1] + (um[2] * t[0] - um[0] * t[2]),
                     um[2] + (um[0] * t[1] - um[1] * t[0])};
    const R d[3] = {(up[1] * sv[2] - up[2] * sv[1]) + (R)2 * h * E[0],
                    (up[2] * sv[0] - up[0] * sv[2]) + (R)2 * h * E[1],
                    (up[0] * sv[1] - up[1] * sv[0]) + (R)2 * h * E[2]};
    o.pn[0] = p0[0] + d[0]; o.pn[1] = p0[1] + d[1]; o.pn[2] = p0[2] + d[2];
    // ---- H_eff (eq:effective_H) from the mean momentum and d, limited
    o.pb[0] = p0[0] + (R)0.5 * d[0]; o.pb[1] = p0[1] + (R)0.5 * d[1]; o.pb[2] = p0[2] + (R)0.5 * d[2];
    o.p2 = o.pb[0] * o.pb[0] + o.pb[1] * o.pb[1] + o.pb[2] * o.pb[2];
    const R cx = diff_of_products(o.pb[1], d[2], o.pb[2], d[1]);
    const R cy = diff_of_products(o.pb[2], d[0], o.pb[0], d[2]);
    const R cz = diff_of_products(o.pb[0], d[1], o.pb[1], d[0]);
    const R c2 = cx * cx + cy * cy + cz * cz;
    const R g_old = sqrt_r<R>((R)1 + p0[0] * p0[0] + p0[1] * p0[1] + p0[2] * p0[2]);
    o.g_new = sqrt_r<R>((R)1 + o.pn[0] * o.pn[0] + o.pn[1] * o.pn[1] + o.pn[2] * o.pn[2]);
    o.gb = (R)0.5 * (g_old + o.g_new);
    o.pbm = sqrt_r<R>(o.p2);
    // H_eff = 0 when the mean momentum vanishes (no direction of motion)
    R ratio = o.p2 > (R)0 ? sqrt_r<R>(c2) * rcp_r<R>(o.p2) : (R)0;
    if (ratio > (R)1) ratio = (R)1;
    o.H = o.p2 > (R)0 ? o.gb * ratio * a.inv_dt : (R)0;
    // A push that is not finite gives H_eff = chi = 0: the particle emits
    // nothing and adds nothing to the ledger; the caller flags it.
    o.bad = !(isfinite(o.pn[0]) && isfinite(o.pn[1]) && isfinite(o.pn[2]) && isfinite(o.H) &&
              isfinite(o.gb));
    if (o.bad) o.H = (R)0;
    o.chi = o.bad ? (R)0 : a.hbar_n * o.H * o.gb;
    return o;
}


template <typename R>
__device__ __forceinline__ R wrap_pos(R v, R L) {
    if (v >= L) v -= L;
    else if (v < (R)0) v += L;
    if (v >= L || v < (R)0) v = (R)0;   // rounding guard (and a corrupt value)
    return v;
}

// The output pointers of the kernel arguments, reached through an opaque copy
// of the argument-segment pointer: the loads happen where they are used.
// The copy names the constant address space, so the fields are read with
// scalar loads.
template <typename R>
__device__ __forceinline__ PhotonOut cold_args() {
    typedef const __attribute__((address_space(4))) char cchar;
    typedef const __attribute__((address_space(4))) PhotonOut cphoton;
    const char *kp = (const char *)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(kp));
    cphoton *q = (cphoton *)((cchar *)kp + offsetof(StepArgs<R>, ph));
    PhotonOut o;
    o.eps = q->eps;
    o.w = q->w;
    for (int c = 0; c < 3; ++c) {
        o.dir[c] = q->dir[c];
        o.pos[c] = q->pos[c];
    }
    o.parent = q->parent;
    o.step = q->step;
    o.k = q->k;
    o.seg_count = q->seg_count;
    o.partials = q->partials;
    return o;
}

// One photon record into slot o of the buffer (section "The field setup":
// photons become particles; direction along the emitter's mean momentum).
__device__ __forceinline__ void store_photon(const PhotonOut &P, uint32_t o, float eps, float w,
                                             const float dir[3], const float pos[3], uint32_t pid,
                                             uint32_t k, uint32_t step) {
    st(P.eps, o, eps);
    st(P.w, o, w);
    st(P.dir[0], o, dir[0]);
    st(P.dir[1], o, dir[1]);
    st(P.dir[2], o, dir[2]);
    if (P.pos[0]) st(P.pos[0], o, pos[0]);
    if (P.pos[1]) st(P.pos[1], o, pos[1]);
    if (P.pos[2]) st(P.pos[2], o, pos[2]);
    st(P.parent, o, pid);
    if (P.k) st(P.k, o, (uint8_t)k);
    if (P.step) st(P.step, o, step);
}

// LDS of the end-of-kernel ledger reduction: every thread's sums.
struct LedgerSmem {
    double d[5][kBlock];
    float f[2][kBlock];
    uint32_t cnt[kWaves];
    uint32_t flags[kWaves];
};

// Partial ledger rows (internal workspace): the SR_LEDGER_COLS columns of a
// ledger row, then the OR of the condition bits of the block (as a double),
// then one pad column.
constexpr int kPartCols = SR_LEDGER_COLS + 2;
constexpr int kPartFlags = SR_LEDGER_COLS;

// LDS of the kernel.  With the MLP sampler: the network, and per wave the
// compacted inputs of the emitted trials and a 16x64 transpose buffer, which
// the ledger reduction reuses after the last round.
template <int KMAX, int SAMPLER, bool BOX = false>
struct alignas(16) StepSmem {
    union {
        struct {
            MlpSmem m;
            alignas(16) float2 io[kWaves][64 * KMAX];
            alignas(16) __bf16 tb[kWaves][2 * 16 * kH];
        };
        LedgerSmem led;
    };
};
// Photons staged in LDS for one block-wide flush: wave w's first kStage photons
// of its (single) round sit at [w][0, kStage).
constexpr int kStage = 64;
struct PhotonStage {
    float eps[kWaves][kStage], w[kWaves][kStage];
    float dir[3][kWaves][kStage], pos[3][kWaves][kStage];
    uint32_t parent[kWaves][kStage], k[kWaves][kStage];
    uint32_t cnt[kWaves];       // staged photons per wave
    uint32_t base[kWaves];      // first buffer slot of each wave's chunk segment
};
// With four or more trials the proposal sampler also keeps the hot pieces of
// the trial-density table in LDS (31.3 KB in all: five 256-thread blocks per
// compute unit), and the quantum sampler those of its kernel table (29.3 KB);
// with fewer trials the table lookups are too few to pay for the copy.
template <int KMAX>
constexpr bool kHotTable = KMAX >= 4;
template <int KMAX>
struct StepSmem<KMAX, SR_SAMPLER_S, false> {
    LedgerSmem led;
    PhotonStage stage;
    float4 ghot[kHotTable<KMAX> ? kGHot : 1];
};
template <int KMAX>
struct StepSmem<KMAX, SR_SAMPLER_TABLE, false> {
    LedgerSmem led;
    PhotonStage stage;
};
template <int KMAX>
struct StepSmem<KMAX, SR_SAMPLER_QUANTUM, false> {
    LedgerSmem led;
    PhotonStage stage;
    float4 qhot[kHotTable<KMAX> ? kQHot : 1];   // 29.3 KB in all
};
// With the LDS field box (SR_GATHER_BOX) the box shares its LDS with the
// ledger and the photon stage: it is read only before either is written.
// 32 352 bytes in all keeps five 256-thread blocks per compute unit.
struct BoxReduce {
    int mn[kWaves][3], mx[kWaves][3];
};
struct alignas(16) BoxSmem {
    union {
        struct {
            LedgerSmem led;
            PhotonStage stage;
        };
        float box[6][kBoxCells];
    };
    BoxReduce red;
};
template <int KMAX>
struct StepSmem<KMAX, SR_SAMPLER_S, true> : BoxSmem {};
template <int KMAX>
struct StepSmem<KMAX, SR_SAMPLER_TABLE, true> : BoxSmem {};
template <int KMAX>
struct StepSmem<KMAX, SR_SAMPLER_QUANTUM, true> : BoxSmem {};
template <typename S>
__device__ __forceinline__ LedgerSmem &ledger_smem(S &s) { return s.led; }

// Field box of a block (3D, uniform chunks, called by every thread of the
// block): the nodes of every stencil of the block's particles, from the
// extremes of their offset-0 base cells widened by one node on each side (the
// offset-1/2 base node is the base cell or the one below it).  A block whose
// cells straddle a periodic boundary, or whose box exceeds kBoxCells nodes or
// wraps onto itself, returns false and gathers directly.  Otherwise the six
// components are copied into LDS with coalesced loads (the caller syncs
// before reading them).
template <typename R>
__device__ __forceinline__ bool load_field_box(const StepArgs<R> &a, BoxSmem &sm, bool act,
                                               const int cell[3], FieldBox &fb) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int lo = wave_min_i(act ? cell[q] : 0x7fffffff);
        const int hi = wave_max_i(act ? cell[q] : -0x7fffffff);
        if (lane == 0) { sm.red.mn[wave][q] = lo; sm.red.mx[wave][q] = hi; }
    }
    __syncthreads();
    int cells = 1;
    bool ok = true;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int lo = min(min(sm.red.mn[0][q], sm.red.mn[1][q]), min(sm.red.mn[2][q], sm.red.mn[3][q]));
        const int hi = max(max(sm.red.mx[0][q], sm.red.mx[1][q]), max(sm.red.mx[2][q], sm.red.mx[3][q]));
        const int n = a.g.n[q];
        const int ext = hi - lo + 3;
        ok = ok && hi >= lo && ext < n;
        fb.lo[q] = lo == 0 ? n - 1 : lo - 1;
        fb.ext[q] = ext;
        cells *= ok ? ext : 1;
    }
    if (!(ok && cells <= kBoxCells)) return false;
    // element e of the box, x fastest; the quotients are exact in binary32
    // (e + 1/2 below 2^22)
    const uint32_t ex = (uint32_t)fb.ext[0], ey = (uint32_t)fb.ext[1];
    const float inv_ex = 1.0f / (float)ex, inv_ey = 1.0f / (float)ey;
    const int nx = a.g.n[0], ny = a.g.n[1], nz = a.g.n[2];
    for (uint32_t e = (uint32_t)tid; e < (uint32_t)cells; e += kBlock) {
        const uint32_t r = (uint32_t)(((float)e + 0.5f) * inv_ex);
        const uint32_t lx = e - r * ex;
        const uint32_t lz = (uint32_t)(((float)r + 0.5f) * inv_ey);
        const uint32_t ly = r - lz * ey;
        int gx = fb.lo[0] + (int)lx, gy = fb.lo[1] + (int)ly, gz = fb.lo[2] + (int)lz;
        gx -= gx >= nx ? nx : 0;
        gy -= gy >= ny ? ny : 0;
        gz -= gz >= nz ? nz : 0;
        const uint32_t off = __umul24(__umul24((uint32_t)gz, (uint32_t)ny) + (uint32_t)gy,
                                      (uint32_t)nx) + (uint32_t)gx;
        float v[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = ld(a.f[c], off);
#pragma unroll
        for (int c = 0; c < 6; ++c) sm.box[c][e] = v[c];
    }
    return true;
}

// Occupancy target: the FP32 3D kernels with 4 to 8 trials sit a couple of
// VGPRs above the 96 that five waves per SIMD allow; asking for five costs no
// spills and gives them a fifth wave.
template <typename R, int DIM, int KMAX, int SAMPLER>
constexpr int step_waves_per_eu() {
    return (sizeof(R) == 4 && DIM == 3 && KMAX >= 4 && KMAX <= 8 && SAMPLER != SR_SAMPLER_MLP) ? 5
                                                                                              : 1;
}

// FLOOR: the grid-frequency floor is on (a.e_grid > 0); a template flag, so the
// kernels without it carry none of its code.
// BOX: the SR_GATHER_BOX gather (3D, uniform chunks, proposal, table or
// quantum sampler); the host launches it only there.
template <typename R, int DIM, int KMAX, int SAMPLER, bool FLOOR, bool BOX>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(step_waves_per_eu<R, DIM, KMAX, SAMPLER>())))
void push_emit_kernel(const StepArgs<R> a) {
    static_assert(!BOX || (DIM == 3 && SAMPLER != SR_SAMPLER_MLP), "the field box is 3D");
    __shared__ StepSmem<KMAX, SAMPLER, BOX> sm;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if constexpr (SAMPLER == SR_SAMPLER_MLP) {
        // the network is copied to LDS only if the fallback map leaves some
        // bin to it (the same decision in every thread of the block)
        bool any_net = false;
        for (int b = 0; b < kMlpFallbackBins; ++b) any_net |= a.mlp_fallback[b] == 0;
        if (any_net) {
            mlp_load(sm.m, a.mlp, tid, kBlock);
            __syncthreads();
        }
    }
    if constexpr (SAMPLER == SR_SAMPLER_S && !BOX && kHotTable<KMAX>) {
        for (int e = tid; e < kGHot; e += kBlock) sm.ghot[e] = a.tab.gtab[ghot_source(e)];
        __syncthreads();
    }
    if constexpr (SAMPLER == SR_SAMPLER_QUANTUM && !BOX && kHotTable<KMAX>) {
        for (int e = tid; e < kQHot; e += kBlock) sm.qhot[e] = a.tab.qtab[2 * kQHot0 + e];
        __syncthreads();
    }
    // one chunk per wave, kWaves consecutive chunks per block (blocks mapped so
    // that neighbouring chunks share an XCD)
    const uint32_t blk = (uint32_t)xcd_chunk(blockIdx.x, gridDim.x);
    const uint32_t c = blk * kWaves + wave;
    const bool have = c < (uint32_t)a.n_chunks;
    // particle and photon counts are below 2^31 (checked on the host)
    uint32_t s0 = 0, e0 = 0;
    if (have) {
        s0 = a.start ? (uint32_t)a.start[c] : c * (uint32_t)kChunk;
        e0 = a.start ? (uint32_t)a.start[c + 1] : min(s0 + (uint32_t)kChunk, (uint32_t)a.n);
    }
    const uint32_t pp = (uint32_t)a.per_particle;
    const uint32_t seg_base = s0 * pp;
    const uint32_t seg_cap = (e0 - s0) * pp;
    // With uniform chunks every wave has a single round, so the S and table
    // samplers stage their photons in LDS and the block writes them together
    // at the end (one store per array for up to 256 photons of four chunks).
    constexpr bool kCanStage = SAMPLER != SR_SAMPLER_MLP;
    const bool staged = kCanStage && a.start == nullptr;
    const int K = a.K;
    const float invK = 1.0f / (float)K;

    // Ledger sums of the lane.  With the proposal and table samplers each
    // round's sums are added to the lane's own LDS ledger slot at the end of
    // the round, so no FP64 sum stays in registers across rounds (it would
    // hold VGPRs through the next round's gather and cost a wave per SIMD);
    // the learned sampler shares that LDS with the network and keeps them in
    // registers.
    constexpr bool kLdsAcc = SAMPLER != SR_SAMPLER_MLP;
    double tot_emit = 0.0, tot_ll = 0.0, tot_de = 0.0, tot_clamp = 0.0, tot_drop = 0.0;
    float tot_w = 0.0f;
    if constexpr (kLdsAcc && !BOX) {
        LedgerSmem &rs = ledger_smem(sm);
#pragma unroll
        for (int q = 0; q < 5; ++q) rs.d[q][tid] = 0.0;
        rs.f[0][tid] = 0.0f;
    }
    float chi_max = 0.0f;
    uint32_t flags = 0;
    uint32_t run_base = 0;
    bool box_used = false;

    // BOX (uniform chunks): exactly one round per wave, waves without a chunk
    // running it with no active lane, so the block-wide steps of the field box
    // are reached by every thread
    for (uint32_t base = s0; BOX ? base == s0 : base < e0; base += kChunk) {
        double acc_emit = 0.0, acc_ll = 0.0, acc_de = 0.0, acc_clamp = 0.0, acc_drop = 0.0;
        float acc_w = 0.0f;
        const uint32_t i = base + lane;
        const bool active = i < e0;
        float eps_unit = 0.0f, wi_f = 0.0f, chif = 0.0f, Hf = 0.0f;
        float dirf[3] = {0.0f, 0.0f, 0.0f}, posf[3] = {0.0f, 0.0f, 0.0f};
        uint32_t pid = 0;
        // state carried from the push to the recoil
        R wi = (R)0, pos[3] = {(R)0, (R)0, (R)0}, pn[3] = {(R)0, (R)0, (R)0};
        R chi = (R)0, gb = (R)1, g_new = (R)1, p2 = (R)0, pbm = (R)0;
        bool bad = false;
        bool use_box = false;
        FieldBox fb{};
        if constexpr (BOX) {
            // positions first: the block's box from its particles' cells
            int cell[3] = {0, 0, 0};
            if (active) {
                pos[0] = ld(a.x[0], i); pos[1] = ld(a.x[1], i); pos[2] = ld(a.x[2], i);
                Axis<R> X, Y, Z;
                setup_axis<R>(a.g, 0, pos[0], X);
                setup_axis<R>(a.g, 1, pos[1], Y);
                setup_axis<R>(a.g, 2, pos[2], Z);
                cell[0] = X.i0; cell[1] = Y.i0; cell[2] = Z.i0;
            }
            use_box = load_field_box<R>(a, sm, active, cell, fb);
            if (use_box) __syncthreads();
            box_used = use_box;
        }
        if (active) {
            wi = ld(a.w, i);
            pid = ld(a.id, i);
            if (!BOX && a.has_pos) {
                pos[0] = ld(a.x[0], i);
                if (DIM != 0 || a.x[1]) pos[1] = ld(a.x[1], i);
                if ((DIM == 3 || DIM == 0) && a.x[2]) pos[2] = ld(a.x[2], i);
            }
            const R p0[3] = {ld(a.p[0], i), ld(a.p[1], i), ld(a.p[2], i)};
            Pushed<R> q;
            if constexpr (BOX) {
                if (use_box) q = push_box<R>(a, pos, p0, sm.box, fb);
                else q = push_heff<R, DIM>(a, pos, p0);
            } else {
                q = push_heff<R, DIM>(a, pos, p0);
            }
            pn[0] = q.pn[0]; pn[1] = q.pn[1]; pn[2] = q.pn[2];
            p2 = q.p2;
            gb = q.gb;
            g_new = q.g_new;
            pbm = q.pbm;
            const R H = q.H;
            chi = q.chi;
            const R pb[3] = {q.pb[0], q.pb[1], q.pb[2]};
            Hf = (float)H;
            chif = (float)chi;
            bad = q.bad;
            if (bad) flags |= SR_W_NONFINITE;
            if (pbm > (R)0) {
                const R inv = rcp_r<R>(pbm);
                dirf[0] = (float)(pb[0] * inv); dirf[1] = (float)(pb[1] * inv);
                dirf[2] = (float)(pb[2] * inv);
            }
            posf[0] = (float)pos[0]; posf[1] = (float)pos[1]; posf[2] = (float)pos[2];
            chi_max = fmaxf(chi_max, chif);
            eps_unit = 1.5f * chif * (float)gb;    // hbar omega_c: photon energy per unit x
            wi_f = (float)wi;
        }
        if constexpr (BOX) {
            if (use_box) __syncthreads();          // every wave is done with the box
            LedgerSmem &rs = ledger_smem(sm);
#pragma unroll
            for (int q = 0; q < 5; ++q) rs.d[q][tid] = 0.0;
            rs.f[0][tid] = 0.0f;
        }

        // ---- K trials.  Inactive lanes take part in the wave-wide steps with a
        // zero rate, so they never emit.  Photon slots: per trial a ballot and the
        // lane prefix (mbcnt); the chunk's segment belongs to this wave alone.
        float delta_ph = 0.0f;                 // sum over trials of frac * eps
        uint32_t wave_tot = 0;
        float2 rr = make_float2(1.0f, 0.0f);
        if (SAMPLER != SR_SAMPLER_S && SAMPLER != SR_SAMPLER_QUANTUM && active && a.kin_cut)
            rr = r_lookup(a.tab.r, chif);
        constexpr bool kProposal = SAMPLER == SR_SAMPLER_S || SAMPLER == SR_SAMPLER_QUANTUM;
        const float rate = !active ? 0.0f : (kProposal ? a.rate_c * Hf : a.direct_c * Hf * rr.x);
        if constexpr (SAMPLER != SR_SAMPLER_MLP) {
            const TrialCut cut = trial_cut(SAMPLER == SR_SAMPLER_S && a.kin_cut != 0, chif);
            // grid cutoff: photons below hbar omega_grid stay with the grid (the
            // S sampler tests it on R', the quantum one on x, the table sampler
            // on the drawn x before the slot is taken)
            TrialCut flr{-__builtin_inff(), __builtin_inff()};
            if (SAMPLER == SR_SAMPLER_S && FLOOR) flr = trial_floor(a.e_grid, eps_unit);
            uint4 words = make_uint4(0, 0, 0, 0);
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                if (k >= uniform_opaque(K)) break;
                if ((k & 1) == 0)
                    words = philox4x32_10(make_uint4(pid, a.step, (uint32_t)(k >> 1), 0u),
                                          a.seed_lo, a.seed_hi);
                const uint32_t wa = (k & 1) ? words.z : words.x;
                const uint32_t wb = (k & 1) ? words.w : words.y;
                float dn = rate, lg = 0.0f, xq = 0.0f;
                bool lower = true;
                if (SAMPLER == SR_SAMPLER_S) {
                    if constexpr (SAMPLER == SR_SAMPLER_S && !BOX && kHotTable<KMAX>)
                        dn = rate * trial_q_hot(wa, a.tab.gtab, sm.ghot, a.tab.pa, lg, lower);
                    else
                        dn = rate * trial_q(wa, a.tab.gtab, a.tab.pa, lg, lower);
                    if (trial_is_cut(cut, lg, lower)) dn = 0.0f;
                    if (FLOOR && trial_is_floored(flr, lg, lower)) dn = 0.0f;
                } else if (SAMPLER == SR_SAMPLER_QUANTUM) {
                    if constexpr (SAMPLER == SR_SAMPLER_QUANTUM && !BOX && kHotTable<KMAX>)
                        dn = rate * quantum_q_t<true>(wa, a.tab.qtab, sm.qhot, a.tab.pa, chif, xq);
                    else
                        dn = rate * quantum_q(wa, a.tab.qtab, a.tab.pa, chif, xq);
                    if (FLOOR && eps_unit * xq < a.e_grid) dn = 0.0f;
                }
                bool emit;
                float frac = invK;
                if (dn >= 1.0f) {
                    emit = true;
                    if (a.dn_policy == SR_DN_WEIGHT) frac = dn * invK;
                } else {
                    emit = wb < (uint32_t)(dn * 4294967296.0f);
                }
                const auto draw_x = [&]() {
                    if (SAMPLER == SR_SAMPLER_S) return trial_x(wa, lg, lower);
                    if (SAMPLER == SR_SAMPLER_QUANTUM) return xq;
                    float lnU, ln1mU;
                    direct_u(wa, rr, lnU, ln1mU);
                    return __builtin_amdgcn_exp2f(t1_log2x(a.tab.t1, lnU, ln1mU));
                };
                float x = 0.0f;
                constexpr bool kDrawFirst = SAMPLER == SR_SAMPLER_TABLE && FLOOR;
                if (kDrawFirst && emit) {
                    x = draw_x();
                    emit = eps_unit * x >= a.e_grid;
                }
                const uint64_t m = __ballot(emit);
                if (m) {
                    if (emit) {
                        if (!kDrawFirst) x = draw_x();
                        const float eps = eps_unit * x;
                        const float wph = wi_f * frac;
                        delta_ph += frac * eps;
                        const uint32_t slot = run_base + wave_tot + lane_prefix(m);
                        if (slot < seg_cap) {
                            if (staged && slot < (uint32_t)kStage) {
                                PhotonStage &S = sm.stage;
                                S.eps[wave][slot] = eps;
                                S.w[wave][slot] = wph;
                                S.dir[0][wave][slot] = dirf[0];
                                S.dir[1][wave][slot] = dirf[1];
                                S.dir[2][wave][slot] = dirf[2];
                                S.pos[0][wave][slot] = posf[0];
                                S.pos[1][wave][slot] = posf[1];
                                S.pos[2][wave][slot] = posf[2];
                                S.parent[wave][slot] = pid;
                                S.k[wave][slot] = (uint32_t)k;
                            } else {
                                store_photon(cold_args<R>(), seg_base + slot, eps, wph, dirf, posf,
                                             pid, (uint32_t)k, a.step);
                            }
                        } else {
                            acc_drop += (double)wph * (double)eps;
                            flags |= SR_W_PHOTON_OVERFLOW;
                        }
                    }
                    wave_tot += (uint32_t)__popcll(m);
                }
            }
        } else {
            // Learned sampler: decisions with the cut rate as for the table; x of
            // the emitted trials from the network, as dense 16-sample tiles on the
            // matrix cores over the wave's compacted trials, except where chi falls
            // in a bin of the fallback map (table instead).
            float2 *io = sm.io[wave];
            const float lchi = (__log2f(fmaxf(chif, 1e-30f)) * 0.30102999566398120f);
            const float fbin = (lchi - kMlpChiLo) * (kMlpFallbackBins / (kMlpChiHi - kMlpChiLo));
            const bool use_table = !active || !(fbin >= 0.0f && fbin < (float)kMlpFallbackBins) ||
                                   a.mlp_fallback[(int)fbin];
            const float f0 = (lchi + 1.0f) * (1.0f / 3.0f);
            uint32_t bits = 0, net_tot = 0;
            float xk[KMAX], fk[KMAX];
            uint32_t off[KMAX], net_off[KMAX];
            uint4 words = make_uint4(0, 0, 0, 0);
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                xk[k] = 0.0f; fk[k] = 0.0f; off[k] = 0; net_off[k] = 0;
                if (k >= K) continue;
                if ((k & 1) == 0)
                    words = philox4x32_10(make_uint4(pid, a.step, (uint32_t)(k >> 1), 0u),
                                          a.seed_lo, a.seed_hi);
                const uint32_t wa = (k & 1) ? words.z : words.x;
                const uint32_t wb = (k & 1) ? words.w : words.y;
                const float dn = rate;
                bool emit;
                float frac = invK;
                if (dn >= 1.0f) {
                    emit = true;
                    if (a.dn_policy == SR_DN_WEIGHT) frac = dn * invK;
                } else {
                    emit = wb < (uint32_t)(dn * 4294967296.0f);
                }
                const uint64_t m = __ballot(emit);
                off[k] = wave_tot + lane_prefix(m);
                wave_tot += (uint32_t)__popcll(m);
                const uint64_t mn = __ballot(emit && !use_table);
                net_off[k] = net_tot + lane_prefix(mn);
                net_tot += (uint32_t)__popcll(mn);
                if (emit) {
                    bits |= 1u << k;
                    fk[k] = frac;
                    if (use_table) {
                        float lnU, ln1mU;
                        direct_u(wa, rr, lnU, ln1mU);
                        xk[k] = __builtin_amdgcn_exp2f(t1_log2x(a.tab.t1, lnU, ln1mU));
                    } else {
                        io[net_off[k]] = make_float2(f0, mlp_feature_u(wa));
                    }
                }
            }
            if (net_tot) {
                wave_lds_sync();
                const int r16 = lane & 15;
                for (uint32_t t0 = 0; t0 < net_tot; t0 += 16) {
                    const uint32_t e = t0 + r16;
                    const float2 f = e < net_tot ? io[e] : make_float2(0.0f, 0.0f);
                    const float y = mlp_tile16(sm.m, sm.tb[wave], f.x, f.y);
                    wave_lds_sync();
                    if (lane < 16 && e < net_tot) io[e].x = y;
                    wave_lds_sync();
                }
                if (!use_table) {
#pragma unroll
                    for (int k = 0; k < KMAX; ++k)
                        if (k < K && ((bits >> k) & 1u))
                            xk[k] = __builtin_amdgcn_exp2f(io[net_off[k]].x);
                }
                wave_lds_sync();
            }
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                if (k < K && ((bits >> k) & 1u)) {
                    const float eps = eps_unit * xk[k];
                    const float wph = wi_f * fk[k];
                    delta_ph += fk[k] * eps;
                    const uint32_t slot = run_base + off[k];
                    if (slot < seg_cap) {
                        store_photon(cold_args<R>(), seg_base + slot, eps, wph, dirf, posf, pid,
                                     (uint32_t)k, a.step);
                    } else {
                        acc_drop += (double)wph * (double)eps;
                        flags |= SR_W_PHOTON_OVERFLOW;
                    }
                }
            }
        }

        if (active) {
            acc_emit += (double)wi_f * (double)delta_ph;
            // Landau-Lifshitz loss of the step (eq:LLformOfRRForce)
            const R beta2 = p2 * rcp_r<R>(gb * gb);
            if (!bad) acc_ll += (double)(wi * a.ll_c * chi * chi * beta2);

            // ---- recoil along the post-push momentum
            R delta = (R)0;
            if (a.recoil == SR_RECOIL_PHOTON) delta = (R)delta_ph;
            else if (a.recoil == SR_RECOIL_LL) delta = a.ll_c * chi * chi * pbm * rcp_r<R>(gb);
            R g_after = g_new;
            if (delta > (R)0) {
                const R pm = sqrt_r<R>(pn[0] * pn[0] + pn[1] * pn[1] + pn[2] * pn[2]);
                R fac = pm > (R)0 ? (R)1 - delta * rcp_r<R>(pm) : (R)-1;
                R removed = delta;
                if (fac < (R)0) {
                    acc_clamp += (double)(wi * (delta - pm));
                    removed = pm;
                    fac = (R)0;
                    flags |= SR_W_RECOIL_CLAMP;
                }
                pn[0] *= fac; pn[1] *= fac; pn[2] *= fac;
                const R pm_after = fac * pm;
                g_after = sqrt_r<R>((R)1 + pm_after * pm_after);
                // gamma_after - gamma_before without cancellation
                acc_de += (double)(-wi * removed * (pm_after + pm) * rcp_r<R>(g_after + g_new));
            }
            if (!(isfinite(pn[0]) && isfinite(pn[1]) && isfinite(pn[2])))
                flags |= SR_W_NONFINITE;
            st(a.p[0], i, pn[0]); st(a.p[1], i, pn[1]); st(a.p[2], i, pn[2]);
            // ---- position push
            if (a.push_position && a.has_pos) {
                const R vdt = a.dt * rcp_r<R>(g_after);
                if (DIM == 0) {
                    st(a.x[0], i, pos[0] + vdt * pn[0]);
                    if (a.x[1]) st(a.x[1], i, pos[1] + vdt * pn[1]);
                    if (a.x[2]) st(a.x[2], i, pos[2] + vdt * pn[2]);
                } else {
                    st(a.x[0], i, wrap_pos<R>(pos[0] + vdt * pn[0], box_len<R>(a.g, 0)));
                    st(a.x[1], i, wrap_pos<R>(pos[1] + vdt * pn[1], box_len<R>(a.g, 1)));
                    if (DIM == 3) st(a.x[2], i, wrap_pos<R>(pos[2] + vdt * pn[2], box_len<R>(a.g, 2)));
                }
            }
            acc_w += wi_f;
        }
        run_base += wave_tot;
        if constexpr (kLdsAcc) {
            LedgerSmem &rs = ledger_smem(sm);
            rs.d[0][tid] += acc_emit;
            rs.d[1][tid] += acc_ll;
            rs.d[2][tid] += acc_de;
            rs.d[3][tid] += acc_clamp;
            rs.d[4][tid] += acc_drop;
            rs.f[0][tid] += acc_w;
        } else {
            tot_emit += acc_emit;
            tot_ll += acc_ll;
            tot_de += acc_de;
            tot_clamp += acc_clamp;
            tot_drop += acc_drop;
            tot_w += acc_w;
        }
    }

    if (have && lane == 0) cold_args<R>().seg_count[c] = run_base;

    // the wave's condition bits; they travel in the block's partial row to the
    // ledger reduction, which latches them into the status word
    uint32_t wf = 0;
    if (__ballot(flags != 0)) {
        wf = flags;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) wf |= (uint32_t)__shfl_xor((int)wf, o, 64);
    }

    // ---- per-block ledger partial (FP64, fixed reduction order).  The lanes'
    // sums go to LDS; then each wave reduces its share of the columns over the
    // whole block (four values per lane, then one wave reduction), so the block
    // pays for each column's wave reduction once.  Clamped and dropped energy
    // are rare: reduced only when some lane has them.
    if constexpr (SAMPLER == SR_SAMPLER_MLP) __syncthreads();   // LDS shared with the sampler
    LedgerSmem &rs = ledger_smem(sm);
    if constexpr (!kLdsAcc) {
        rs.d[0][tid] = tot_emit;
        rs.d[1][tid] = tot_ll;
        rs.d[2][tid] = tot_de;
        rs.d[3][tid] = tot_clamp;
        rs.d[4][tid] = tot_drop;
        rs.f[0][tid] = tot_w;
    }
    rs.f[1][tid] = chi_max;
    if (lane == 0) {
        rs.cnt[wave] = run_base;
        rs.flags[wave] = wf;
    }
    if constexpr (kCanStage) {
        if (staged && lane == 0) {
            sm.stage.cnt[wave] = min(min(run_base, seg_cap), (uint32_t)kStage);
            sm.stage.base[wave] = seg_base;
        }
    }
    __syncthreads();
    if constexpr (kCanStage) {
        if (staged) {
            const PhotonStage &S = sm.stage;
            const uint32_t c0 = S.cnt[0], c1 = c0 + S.cnt[1], c2 = c1 + S.cnt[2];
            const uint32_t total = c2 + S.cnt[3];
            const uint32_t e = (uint32_t)tid;
            if (e < total) {
                const int wv = (int)(e >= c0) + (int)(e >= c1) + (int)(e >= c2);
                const uint32_t j = e - (wv == 0 ? 0u : wv == 1 ? c0 : wv == 2 ? c1 : c2);
                const float d[3] = {S.dir[0][wv][j], S.dir[1][wv][j], S.dir[2][wv][j]};
                const float ps[3] = {S.pos[0][wv][j], S.pos[1][wv][j], S.pos[2][wv][j]};
                store_photon(cold_args<R>(), S.base[wv] + j, S.eps[wv][j], S.w[wv][j], d, ps,
                             S.parent[wv][j], S.k[wv][j], a.step);
            }
        }
    }
    double *row = cold_args<R>().partials + (size_t)blk * kPartCols;
    const auto dsum = [&](int q) {
        const double v = ((rs.d[q][lane] + rs.d[q][lane + 64]) + rs.d[q][lane + 128]) +
                         rs.d[q][lane + 192];
        return __ballot(v != 0.0) ? wave_sum(v) : 0.0;
    };
    if (wave == 0) {
        const double e = dsum(0), dr = dsum(4);
        if (lane == 0) { row[SR_LED_EMITTED] = e; row[SR_LED_DROPPED] = dr; }
    } else if (wave == 1) {
        const double l = dsum(1);
        const float m = wave_max(fmaxf(fmaxf(rs.f[1][lane], rs.f[1][lane + 64]),
                                       fmaxf(rs.f[1][lane + 128], rs.f[1][lane + 192])));
        if (lane == 0) { row[SR_LED_LL] = l; row[SR_LED_CHI_MAX] = (double)m; }
    } else if (wave == 2) {
        const double de = dsum(2);
        const float w = wave_sum_f(((rs.f[0][lane] + rs.f[0][lane + 64]) + rs.f[0][lane + 128]) +
                                   rs.f[0][lane + 192]);
        if (lane == 0) { row[SR_LED_RECOIL] = de; row[SR_LED_WEIGHT] = (double)w; }
    } else {
        const double cl = dsum(3);
        if (lane == 0) {
            row[SR_LED_CLAMPED] = cl;
            row[SR_LED_PHOTONS] = (double)((rs.cnt[0] + rs.cnt[1]) + (rs.cnt[2] + rs.cnt[3]));
            row[kPartFlags] = (double)(rs.flags[0] | rs.flags[1] | rs.flags[2] | rs.flags[3]);
            // the last column marks the blocks that gathered from the field box
            row[kPartFlags + 1] = box_used ? 1.0 : 0.0;
        }
    }
}

// Sum partial rows [lo, hi) of `in` (column SR_LED_CHI_MAX is a maximum, the
// flags column an OR).  Each thread keeps all columns of a strided set of rows
// in registers, then the block combines them with wave shuffles and LDS: a
// fixed order, so the ledger is bit-reproducible.  With status == nullptr the
// block writes the partial row out[0..kPartCols); otherwise it writes the
// ledger row out[0..SR_LEDGER_COLS) and ORs the flags into *status (one atomic
// per reduction).  Call with the whole block.
__device__ __forceinline__ void ledger_sum_block(const double *__restrict__ in, int64_t lo,
                                                 int64_t hi, double *__restrict__ out,
                                                 uint32_t *__restrict__ status) {
    __shared__ double s[kWaves][SR_LEDGER_COLS];
    __shared__ uint32_t sf[kWaves];
    double acc[SR_LEDGER_COLS];
    uint32_t fl = 0;
#pragma unroll
    for (int c = 0; c < SR_LEDGER_COLS; ++c) acc[c] = 0.0;
    for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) {
        const double2 *row = (const double2 *)(in + r * kPartCols);
#pragma unroll
        for (int q = 0; q < SR_LEDGER_COLS / 2; ++q) {
            const double2 v = row[q];
            const int c0 = 2 * q, c1 = 2 * q + 1;
            acc[c0] = c0 == SR_LED_CHI_MAX ? fmax(acc[c0], v.x) : acc[c0] + v.x;
            acc[c1] = c1 == SR_LED_CHI_MAX ? fmax(acc[c1], v.y) : acc[c1] + v.y;
        }
        fl |= (uint32_t)row[kPartFlags / 2].x;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < SR_LEDGER_COLS; ++c) {
        double v = acc[c];
        for (int o = 32; o > 0; o >>= 1) {
            const double u = __shfl_xor(v, o, 64);
            v = c == SR_LED_CHI_MAX ? fmax(v, u) : v + u;
        }
        if (lane == 0) s[wave][c] = v;
    }
    for (int o = 32; o > 0; o >>= 1) fl |= (uint32_t)__shfl_xor((int)fl, o, 64);
    if (lane == 0) sf[wave] = fl;
    __syncthreads();
    if (threadIdx.x < SR_LEDGER_COLS) {
        const int c = threadIdx.x;
        double v = s[0][c];
        for (int w = 1; w < kWaves; ++w) v = c == SR_LED_CHI_MAX ? fmax(v, s[w][c]) : v + s[w][c];
        out[c] = v;
    } else if (threadIdx.x == SR_LEDGER_COLS) {
        uint32_t f = 0;
        for (int w = 0; w < kWaves; ++w) f |= sf[w];
        if (status) {
            if (f) atomicOr(status, f);
        } else {
            out[kPartFlags] = (double)f;
            out[kPartFlags + 1] = 0.0;
        }
    }
}

// Block b sums rows [b per, (b + 1) per) of the n_rows rows of `in`: into
// partial row out[b] (status == nullptr), or, as the only block, into the
// ledger row out.
__global__ __launch_bounds__(kBlock) void ledger_reduce_kernel(const double *__restrict__ in,
                                                               int64_t n_rows, int64_t per_block,
                                                               double *__restrict__ out,
                                                               uint32_t *__restrict__ status) {
    const int64_t lo = (int64_t)blockIdx.x * per_block;
    const int64_t hi = min(lo + per_block, n_rows);
    ledger_sum_block(in, lo, hi, status ? out : out + (int64_t)blockIdx.x * kPartCols, status);
}

// partial ledger rows written by one step: one per block of kWaves chunks
inline int64_t partial_rows(int64_t n_chunks) { return (n_chunks + kWaves - 1) / kWaves; }

__global__ void zero_row_kernel(double *row) {
    if (threadIdx.x < SR_LEDGER_COLS) row[threadIdx.x] = 0.0;
}

constexpr int64_t kReduceL1Blocks = 1024;
constexpr int64_t kReduceSingle = 512;     // rows one block sums directly
constexpr int64_t kReducePerBlock = 64;    // rows per block in the first of two levels

// How one step's partial rows are summed: none (a zero row), by one block, or
// in two levels (first-level rows in the partials buffer after the step's).
struct LedgerPlan {
    int mode;          // 0 zero row, 1 one block, 2 two levels
    int64_t rows;      // partial rows of the step
    int64_t per, nb;   // two levels: rows per first-level block, blocks
    double *dst, *mid;
};

LedgerPlan ledger_plan(const sr_ledger *led, int64_t n_chunks, int64_t row) {
    LedgerPlan p;
    p.dst = led->rows + row * SR_LEDGER_COLS;
    p.rows = partial_rows(n_chunks);   // the step writes one partial row per block
    p.per = p.rows;
    p.nb = 1;
    p.mid = nullptr;
    p.mode = p.rows == 0 ? 0 : (p.rows <= kReduceSingle ? 1 : 2);
    if (p.mode == 2) {
        p.per = (p.rows + kReduceL1Blocks - 1) / kReduceL1Blocks;
        if (p.per < kReducePerBlock) p.per = kReducePerBlock;
        p.nb = (p.rows + p.per - 1) / p.per;
        p.mid = led->partials + p.rows * kPartCols;
    }
    return p;
}

int reduce_ledger(const sr_ledger *led, int64_t n_chunks, int64_t row, hipStream_t st) {
    const LedgerPlan p = ledger_plan(led, n_chunks, row);
    if (p.mode == 0) {
        zero_row_kernel<<<1, 64, 0, st>>>(p.dst);
    } else if (p.mode == 1) {
        ledger_reduce_kernel<<<1, kBlock, 0, st>>>(led->partials, p.rows, p.rows, p.dst,
                                                   led->status);
    } else {
        ledger_reduce_kernel<<<(unsigned)p.nb, kBlock, 0, st>>>(led->partials, p.rows, p.per,
                                                                p.mid, nullptr);
        ledger_reduce_kernel<<<1, kBlock, 0, st>>>(p.mid, p.nb, p.nb, p.dst, led->status);
    }
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

// Step epilogue, first launch: blocks [0, nb_led) do the ledger's only or
// first level (n_rows == 0: block 0 writes a zero row), the other nb_hist
// blocks accumulate the photon spectrum.
__global__ __launch_bounds__(kBlock) void epilogue_first_kernel(
    const double *__restrict__ in, int64_t n_rows, int64_t per, int nb_led,
    double *__restrict__ out, uint32_t *__restrict__ status, sr_photon_buf ph,
    const int64_t *start, int64_t n_chunks, int64_t n, float l2lo, float scale, int nbins,
    double *__restrict__ work, int nb_hist) {
    extern __shared__ double sh[];   // [2*nbins], histogram blocks
    const int b = blockIdx.x;
    if (b < nb_led) {
        if (n_rows == 0) {
            if (threadIdx.x < SR_LEDGER_COLS) out[threadIdx.x] = 0.0;
            return;
        }
        const int64_t lo = (int64_t)b * per;
        const int64_t hi = min(lo + per, n_rows);
        ledger_sum_block(in, lo, hi, status ? out : out + (int64_t)b * kPartCols, status);
        return;
    }
    hist_block(ph, start, n_chunks, n, l2lo, scale, nbins, work, b - nb_led, nb_hist, sh);
}

// Second launch: with led_blocks = 1, block 0 sums the ledger's first-level
// rows into the ledger row; the other blocks each reduce one histogram value.
__global__ __launch_bounds__(kBlock) void epilogue_second_kernel(
    const double *__restrict__ mid, int64_t nb_mid, double *__restrict__ dst,
    uint32_t *__restrict__ status, int led_blocks, const double *__restrict__ work, int nb_hist,
    int nvals, double *__restrict__ hist) {
    if ((int)blockIdx.x < led_blocks) {
        ledger_sum_block(mid, 0, nb_mid, dst, status);
        return;
    }
    hist_reduce_value(work, nb_hist, nvals, hist, (int)blockIdx.x - led_blocks);
}

// ---------------------------------------------------------------------------
// Many steps in one launch in a uniform field (no grid): every particle's state
// stays in registers across the steps, one wave per block.  Per step: the push
// and H_eff (eq:effective_H), the K trials of section "Monte Carlo method",
// photon append into the chunk's segment (shared by all the steps of the
// launch, each record tagged with its step), recoil and position; each wave
// writes one partial ledger row per step (partials[s][wave]), which
// steps_reduce_kernel sums per step in a fixed order.
template <int KMAX, int SAMPLER>
__global__ __launch_bounds__(64) void push_emit_steps_kernel(const StepArgs<float> a,
                                                             int64_t n_steps) {
    const int lane = threadIdx.x;
    const uint32_t c = blockIdx.x;                      // chunk = wave = block
    const uint32_t s0 = c * (uint32_t)kChunk;
    const uint32_t e0 = min(s0 + (uint32_t)kChunk, (uint32_t)a.n);
    const uint32_t i = s0 + lane;
    const bool active = i < e0;
    const uint32_t pp = (uint32_t)a.per_particle;
    const uint32_t seg_base = s0 * pp, seg_cap = (e0 - s0) * pp;
    const PhotonOut P = cold_args<float>();
    const int K = a.K;
    const float invK = 1.0f / (float)K;
    const int64_t nb = gridDim.x;

    float wi = 0.0f, pos[3] = {0.0f, 0.0f, 0.0f}, p[3] = {0.0f, 0.0f, 0.0f};
    uint32_t pid = 0;
    if (active) {
        wi = ld(a.w, i);
        pid = ld(a.id, i);
        if (a.has_pos) {
            pos[0] = ld(a.x[0], i);
            if (a.x[1]) pos[1] = ld(a.x[1], i);
            if (a.x[2]) pos[2] = ld(a.x[2], i);
        }
        p[0] = ld(a.p[0], i); p[1] = ld(a.p[1], i); p[2] = ld(a.p[2], i);
    }
    const float E[3] = {a.g.e0[0], a.g.e0[1], a.g.e0[2]};
    const float B[3] = {a.g.b0[0], a.g.b0[1], a.g.b0[2]};
    uint32_t run_base = 0;
    for (int64_t si = 0; si < n_steps; ++si) {
        const uint32_t step = a.step + (uint32_t)si;
        double acc_emit = 0.0, acc_ll = 0.0, acc_de = 0.0, acc_clamp = 0.0, acc_drop = 0.0;
        float chif = 0.0f, eps_unit = 0.0f, Hf = 0.0f, dirf[3] = {0.0f, 0.0f, 0.0f};
        float pn[3] = {p[0], p[1], p[2]}, gb = 1.0f, g_new = 1.0f, p2 = 0.0f, pbm = 0.0f,
              chi = 0.0f;
        uint32_t flags = 0;
        bool bad = false;
        if (active) {
            const Pushed<float> q = push_fields<float>(a, p, E, B);
            pn[0] = q.pn[0]; pn[1] = q.pn[1]; pn[2] = q.pn[2];
            p2 = q.p2; gb = q.gb; g_new = q.g_new; pbm = q.pbm; chi = q.chi;
            Hf = q.H;
            chif = q.chi;
            bad = q.bad;
            if (bad) flags |= SR_W_NONFINITE;
            if (pbm > 0.0f) {
                const float inv = rcp_r<float>(pbm);
                dirf[0] = q.pb[0] * inv; dirf[1] = q.pb[1] * inv; dirf[2] = q.pb[2] * inv;
            }
            eps_unit = 1.5f * chif * gb;
        }
        float delta_ph = 0.0f;
        uint32_t wave_tot = 0;
        float2 rr = make_float2(1.0f, 0.0f);
        if (SAMPLER == SR_SAMPLER_TABLE && active && a.kin_cut) rr = r_lookup(a.tab.r, chif);
        constexpr bool kProposal = SAMPLER == SR_SAMPLER_S || SAMPLER == SR_SAMPLER_QUANTUM;
        const float rate = !active ? 0.0f : (kProposal ? a.rate_c * Hf : a.direct_c * Hf * rr.x);
        const TrialCut cut = trial_cut(SAMPLER == SR_SAMPLER_S && a.kin_cut != 0, chif);
        uint4 words = make_uint4(0, 0, 0, 0);
        for (int k = 0; k < KMAX; ++k) {
            if (k >= K) break;
            if ((k & 1) == 0)
                words = philox4x32_10(make_uint4(pid, step, (uint32_t)(k >> 1), 0u), a.seed_lo,
                                      a.seed_hi);
            const uint32_t wa = (k & 1) ? words.z : words.x;
            const uint32_t wb = (k & 1) ? words.w : words.y;
            float dn = rate, lg = 0.0f, xq = 0.0f;
            bool lower = true;
            if (SAMPLER == SR_SAMPLER_S) {
                dn = rate * trial_q(wa, a.tab.gtab, a.tab.pa, lg, lower);
                if (trial_is_cut(cut, lg, lower)) dn = 0.0f;
            } else if (SAMPLER == SR_SAMPLER_QUANTUM) {
                dn = rate * quantum_q(wa, a.tab.qtab, a.tab.pa, chif, xq);
            }
            bool emit;
            float frac = invK;
            if (dn >= 1.0f) {
                emit = true;
                if (a.dn_policy == SR_DN_WEIGHT) frac = dn * invK;
            } else {
                emit = wb < (uint32_t)(dn * 4294967296.0f);
            }
            const uint64_t m = __ballot(emit);
            if (m) {
                if (emit) {
                    float x;
                    if (SAMPLER == SR_SAMPLER_S) {
                        x = trial_x(wa, lg, lower);
                    } else if (SAMPLER == SR_SAMPLER_QUANTUM) {
                        x = xq;
                    } else {
                        float lnU, ln1mU;
                        direct_u(wa, rr, lnU, ln1mU);
                        x = __builtin_amdgcn_exp2f(t1_log2x(a.tab.t1, lnU, ln1mU));
                    }
                    const float eps = eps_unit * x;
                    const float wph = wi * frac;
                    delta_ph += frac * eps;
                    const uint32_t slot = run_base + wave_tot + lane_prefix(m);
                    if (slot < seg_cap) {
                        store_photon(P, seg_base + slot, eps, wph, dirf, pos, pid, (uint32_t)k, step);
                    } else {
                        acc_drop += (double)wph * (double)eps;
                        flags |= SR_W_PHOTON_OVERFLOW;
                    }
                }
                wave_tot += (uint32_t)__popcll(m);
            }
        }
        float acc_w = 0.0f;
        if (active) {
            acc_emit = (double)wi * (double)delta_ph;
            const float beta2 = p2 * rcp_r<float>(gb * gb);
            if (!bad) acc_ll = (double)(wi * a.ll_c * chi * chi * beta2);
            float delta = 0.0f;
            if (a.recoil == SR_RECOIL_PHOTON) delta = delta_ph;
            else if (a.recoil == SR_RECOIL_LL) delta = a.ll_c * chi * chi * pbm * rcp_r<float>(gb);
            float g_after = g_new;
            if (delta > 0.0f) {
                const float pm = sqrt_r<float>(pn[0] * pn[0] + pn[1] * pn[1] + pn[2] * pn[2]);
                float fac = pm > 0.0f ? 1.0f - delta * rcp_r<float>(pm) : -1.0f;
                float removed = delta;
                if (fac < 0.0f) {
                    acc_clamp = (double)(wi * (delta - pm));
                    removed = pm;
                    fac = 0.0f;
                    flags |= SR_W_RECOIL_CLAMP;
                }
                pn[0] *= fac; pn[1] *= fac; pn[2] *= fac;
                const float pm_after = fac * pm;
                g_after = sqrt_r<float>(1.0f + pm_after * pm_after);
                acc_de = (double)(-wi * removed * (pm_after + pm) * rcp_r<float>(g_after + g_new));
            }
            if (!(isfinite(pn[0]) && isfinite(pn[1]) && isfinite(pn[2]))) flags |= SR_W_NONFINITE;
            if (a.push_position && a.has_pos) {
                const float vdt = a.dt * rcp_r<float>(g_after);
                pos[0] += vdt * pn[0]; pos[1] += vdt * pn[1]; pos[2] += vdt * pn[2];
            }
            p[0] = pn[0]; p[1] = pn[1]; p[2] = pn[2];
            acc_w = wi;
        }
        run_base += wave_tot;
        // this wave's partial ledger row of the step (fixed-order wave sums)
        const double se = wave_sum(acc_emit), sl = wave_sum(acc_ll), sd = wave_sum(acc_de);
        const double sc = __ballot(acc_clamp != 0.0) ? wave_sum(acc_clamp) : 0.0;
        const double sdr = __ballot(acc_drop != 0.0) ? wave_sum(acc_drop) : 0.0;
        const float sw = wave_sum_f(acc_w), cm = wave_max(chif);
        uint32_t wf = 0;
        if (__ballot(flags != 0)) {
            wf = flags;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) wf |= (uint32_t)__shfl_xor((int)wf, o, 64);
        }
        if (lane == 0) {
            double *row = P.partials + (si * nb + c) * kPartCols;
            row[SR_LED_EMITTED] = se;
            row[SR_LED_LL] = sl;
            row[SR_LED_RECOIL] = sd;
            row[SR_LED_CLAMPED] = sc;
            row[SR_LED_DROPPED] = sdr;
            row[SR_LED_PHOTONS] = (double)wave_tot;
            row[SR_LED_WEIGHT] = (double)sw;
            row[SR_LED_CHI_MAX] = (double)cm;
            row[kPartFlags] = (double)wf;
            row[kPartFlags + 1] = 0.0;
        }
    }
    if (active) {
        st(a.p[0], i, p[0]); st(a.p[1], i, p[1]); st(a.p[2], i, p[2]);
        if (a.push_position && a.has_pos) {
            st(a.x[0], i, pos[0]);
            if (a.x[1]) st(a.x[1], i, pos[1]);
            if (a.x[2]) st(a.x[2], i, pos[2]);
        }
    }
    if (lane == 0) P.seg_count[c] = run_base;
}

// Ledger row s of a multi-step launch: the nb partial rows of step s, summed in
// a fixed order, with the condition bits latched into *status.
__global__ __launch_bounds__(kBlock) void steps_reduce_kernel(const double *__restrict__ partials,
                                                              int64_t nb, double *__restrict__ rows,
                                                              uint32_t *__restrict__ status) {
    const int64_t s = blockIdx.x;
    ledger_sum_block(partials + s * nb * kPartCols, 0, nb, rows + s * SR_LEDGER_COLS, status);
}

void split_inv(double dx, float &hi, float &lo) {
    const double inv = 1.0 / dx;
    hi = (float)inv;
    lo = (float)(inv - (double)hi);
}

// Validation and kernel arguments shared by the step and the push evaluation:
// particles, grid, fields, dt and the physical constants of prm.
template <typename R, typename PARTS>
int particle_args(PARTS *parts, const sr_fields_f32 *fields, const sr_grid *grid, double dt,
                  const sr_params *prm, StepArgs<R> &a) {
    if (!parts || !grid || !prm) return SR_E_INVAL;
    const int64_t n = parts->n;
    if (n < 0 || !(dt > 0.0)) return SR_E_INVAL;
    if (!(prm->hbar_n > 0.0) || !(prm->alpha > 0.0)) return SR_E_INVAL;
    const int dim = grid->dim;
    if (dim != 0 && dim != 2 && dim != 3) return SR_E_INVAL;
    // the kernels address every array with 32-bit byte offsets
    if (n >= ((int64_t)1 << 31) / (int64_t)sizeof(R)) return SR_E_UNSUPPORTED;
    if (n > 0 && (!parts->p[0] || !parts->p[1] || !parts->p[2] || !parts->w || !parts->id))
        return SR_E_INVAL;
    const bool has_pos = parts->x[0] != nullptr;
    if (dim != 0) {
        if (!fields) return SR_E_INVAL;
        for (int q = 0; q < 3; ++q)
            if (!fields->e[q] || !fields->b[q]) return SR_E_INVAL;
        if (n > 0 && (!parts->x[0] || !parts->x[1] || (dim == 3 && !parts->x[2])))
            return SR_E_INVAL;
        for (int q = 0; q < dim; ++q)
            if (grid->n[q] < 1 || grid->n[q] > (1 << 24) || !(grid->dx[q] > 0.0)) return SR_E_INVAL;
        if (grid->n[0] < 2) return SR_E_INVAL;   // rows are read as pairs
        if (grid->n[1] * (dim == 3 ? grid->n[2] : 1) >= ((int64_t)1 << 24)) return SR_E_UNSUPPORTED;
        if (dim == 2 && grid->n[2] != 1) return SR_E_INVAL;
        const int64_t cells = grid->n[0] * grid->n[1] * (dim == 3 ? grid->n[2] : 1);
        if (cells <= 0) return SR_E_INVAL;
        if (cells >= ((int64_t)1 << 30)) return SR_E_UNSUPPORTED;
    }
    a.n = n;
    for (int q = 0; q < 3; ++q) { a.x[q] = parts->x[q]; a.p[q] = parts->p[q]; }
    a.w = parts->w;
    a.id = parts->id;
    for (int q = 0; q < 3; ++q) {
        a.f[q] = fields ? fields->e[q] : nullptr;
        a.f[3 + q] = fields ? fields->b[q] : nullptr;
    }
    GridK &g = a.g;
    g.dim = dim;
    for (int q = 0; q < 3; ++q) {
        g.n[q] = (int)(dim == 0 ? 1 : grid->n[q]);
        const double dxq = dim == 0 ? 1.0 : grid->dx[q];
        split_inv(dxq, g.inv_hi[q], g.inv_lo[q]);
        g.inv_d[q] = 1.0 / dxq;
        g.Ld[q] = (double)g.n[q] * dxq;
        g.L[q] = (float)g.Ld[q];
        g.e0[q] = (float)grid->e0[q];
        g.b0[q] = (float)grid->b0[q];
        g.e0d[q] = grid->e0[q];
        g.b0d[q] = grid->b0[q];
    }
    if (dim == 2) { g.n[2] = 1; }
    a.dt = (R)dt;
    a.inv_dt = (R)(1.0 / dt);
    a.has_pos = has_pos ? 1 : 0;
    a.hbar_n = (R)prm->hbar_n;
    a.rate_c = (float)(dt * 1.7320508075688772 / (2.0 * 3.14159265358979323846) * prm->alpha);
    a.direct_c = (float)(dt * 5.0 / (2.0 * 1.7320508075688772) * prm->alpha);
    a.ll_c = (R)((2.0 / 3.0) * (prm->alpha / prm->hbar_n) * dt);
    a.e_grid = (float)(prm->hbar_n * prm->omega_grid);
    return SR_OK;
}

template <typename R, typename PARTS>
int prepare_step(PARTS *parts, const sr_fields_f32 *fields, const sr_grid *grid, double dt,
                 uint64_t seed, uint64_t step, const sr_params *prm, const sr_table *tab,
                 const sr_chunking *chunks, sr_photon_buf *ph, sr_ledger *led, bool one_step,
                 StepArgs<R> &a, int64_t &n_chunks_out) {
    if (!parts || !grid || !prm || !tab || !chunks || !ph || !led) return SR_E_INVAL;
    const int rc = particle_args<R>(parts, fields, grid, dt, prm, a);
    if (rc != SR_OK) return rc;
    const int64_t n = parts->n;
    const int dim = grid->dim;
    const int K = prm->n_samples;
    if (K < 1 || K > kMaxK) return SR_E_INVAL;
    if (prm->sampler < SR_SAMPLER_S || prm->sampler > SR_SAMPLER_QUANTUM) return SR_E_INVAL;
    if (prm->sampler == SR_SAMPLER_MLP && (!prm->mlp_params || !prm->mlp_fallback))
        return SR_E_INVAL;
    // the grid floor needs x before the slot is taken; the learned sampler finds
    // x after it
    if (!(prm->omega_grid >= 0.0) || !isfinite(prm->omega_grid)) return SR_E_INVAL;
    if (prm->sampler == SR_SAMPLER_MLP && prm->omega_grid > 0.0) return SR_E_INVAL;
    if (prm->recoil < 0 || prm->recoil > 2 || prm->dn_policy < 0 || prm->dn_policy > 1)
        return SR_E_INVAL;
    if (prm->gather != SR_GATHER_DIRECT && prm->gather != SR_GATHER_BOX) return SR_E_INVAL;
    const int64_t n_chunks = chunks->start ? chunks->n_chunks : (n + kChunk - 1) / kChunk;
    if (chunks->start == nullptr && chunks->n_chunks != n_chunks) return SR_E_INVAL;
    if (n_chunks < 0 || n_chunks > 0x7FFFFFFF) return SR_E_INVAL;
    if (ph->per_particle < 0 || !ph->seg_count) return SR_E_INVAL;
    if (n * ph->per_particle >= ((int64_t)1 << 30)) return SR_E_UNSUPPORTED;
    if (ph->per_particle > 0 &&
        (!ph->eps || !ph->w || !ph->dir[0] || !ph->dir[1] || !ph->dir[2] || !ph->parent))
        return SR_E_INVAL;
    if (!led->partials || !led->status) return SR_E_INVAL;
    if (one_step && led->partials_len < sr_ledger_partials(n_chunks)) return SR_E_INVAL;
    n_chunks_out = n_chunks;

    a.seed_lo = (uint32_t)seed;
    a.seed_hi = (uint32_t)(seed >> 32);
    a.step = (uint32_t)step;
    a.K = K;
    a.recoil = prm->recoil;
    a.dn_policy = prm->dn_policy;
    a.kin_cut = prm->kin_cut;
    a.push_position = prm->push_position;
    a.tab.ftab = tab->ftab;
    a.tab.pa = tab->pa;
    a.tab.t1 = tab->t1;
    a.tab.r = tab->r;
    a.tab.gtab = tab->gtab;
    a.tab.qtab = tab->qtab;
    a.mlp = (const __bf16 *)prm->mlp_params;
    a.mlp_fallback = prm->mlp_fallback;
    a.start = chunks->start;
    a.n_chunks = n_chunks;
    a.per_particle = ph->per_particle;
    a.ph.seg_count = ph->seg_count;
    a.ph.eps = ph->eps;
    a.ph.w = ph->w;
    for (int q = 0; q < 3; ++q) { a.ph.dir[q] = ph->dir[q]; a.ph.pos[q] = ph->pos[q]; }
    a.ph.parent = ph->parent;
    a.ph.k = ph->k;
    a.ph.step = ph->step;
    a.ph.partials = led->partials;
    return SR_OK;
}

template <typename R, typename PARTS>
int launch_step(PARTS *parts, const sr_fields_f32 *fields, const sr_grid *grid, double dt,
                uint64_t seed, uint64_t step, const sr_params *prm, const sr_table *tab,
                const sr_chunking *chunks, sr_photon_buf *ph, sr_ledger *led, void *stream,
                void *ev_start = nullptr, void *ev_stop = nullptr) {
    StepArgs<R> a;
    int64_t n_chunks = 0;
    const int rc = prepare_step<R>(parts, fields, grid, dt, seed, step, prm, tab, chunks, ph, led,
                                   true, a, n_chunks);
    if (rc != SR_OK) return rc;
    if (n_chunks == 0) return SR_OK;
    const int dim = grid->dim;
    const int K = prm->n_samples;

    hipStream_t st = (hipStream_t)stream;
    const dim3 grd((unsigned)partial_rows(n_chunks)), blk(kBlock);
    const int KM = K <= 1 ? 1 : K <= 2 ? 2 : K <= 4 ? 4 : K <= 8 ? 8 : 16;

    // with events: the dispatch packet itself records the kernel's start and stop
    // the field-box gather: FP32 path, 3D, uniform chunks, not the learned sampler
    constexpr bool kBoxR = std::is_same<R, float>::value;
    const bool box = prm->gather == SR_GATHER_BOX && dim == 3 && chunks->start == nullptr &&
                     prm->sampler != SR_SAMPLER_MLP;
#define SR_LAUNCH(DIMV, KMV, SMP, FL, BX)                                                      \
    if (ev_start || ev_stop)                                                                   \
        hipExtLaunchKernelGGL(push_emit_kernel<R, DIMV, KMV, SMP, FL, BX>, grd, blk, 0, st,    \
                              (hipEvent_t)ev_start, (hipEvent_t)ev_stop, 0, a);                \
    else                                                                                       \
        push_emit_kernel<R, DIMV, KMV, SMP, FL, BX><<<grd, blk, 0, st>>>(a)
#define SR_BY_K(DIMV, SMP, FL, BX)                         \
    switch (KM) {                                          \
        case 1: SR_LAUNCH(DIMV, 1, SMP, FL, BX); break;    \
        case 2: SR_LAUNCH(DIMV, 2, SMP, FL, BX); break;    \
        case 4: SR_LAUNCH(DIMV, 4, SMP, FL, BX); break;    \
        case 8: SR_LAUNCH(DIMV, 8, SMP, FL, BX); break;    \
        default: SR_LAUNCH(DIMV, 16, SMP, FL, BX); break;  \
    }
#define SR_BY_DIM(SMP, FL, BOXOK)                                      \
    switch (dim) {                                                     \
        case 0: SR_BY_K(0, SMP, FL, false); break;                     \
        case 2: SR_BY_K(2, SMP, FL, false); break;                     \
        default:                                                       \
            if (box) { SR_BY_K(3, SMP, FL, (BOXOK && kBoxR)); }        \
            else { SR_BY_K(3, SMP, FL, false); }                       \
            break;                                                     \
    }
#define SR_BY_FLOOR(SMP)                                     \
    if (a.e_grid > 0.0f) { SR_BY_DIM(SMP, true, true); }     \
    else { SR_BY_DIM(SMP, false, true); }
    if (prm->sampler == SR_SAMPLER_S) { SR_BY_FLOOR(SR_SAMPLER_S); }
    else if (prm->sampler == SR_SAMPLER_TABLE) { SR_BY_FLOOR(SR_SAMPLER_TABLE); }
    else if (prm->sampler == SR_SAMPLER_QUANTUM) { SR_BY_FLOOR(SR_SAMPLER_QUANTUM); }
    else { SR_BY_DIM(SR_SAMPLER_MLP, false, false); }
#undef SR_BY_FLOOR
#undef SR_BY_DIM
#undef SR_BY_K
#undef SR_LAUNCH
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

// Ledger partials for a multi-step launch over n_chunks chunks (doubles).
inline int64_t steps_partials(int64_t n_chunks, int64_t n_steps) {
    return n_steps * n_chunks * kPartCols;
}

int launch_steps(sr_particles_f32 *parts, const sr_grid *grid, double dt, uint64_t seed,
                 uint64_t step0, int64_t n_steps, const sr_params *prm, const sr_table *tab,
                 sr_photon_buf *ph, sr_ledger *led, void *stream) {
    if (!parts || !grid || !prm || !tab || !ph || !led) return SR_E_INVAL;
    if (n_steps < 1 || n_steps > 0x7FFFFFFF) return SR_E_INVAL;
    if (grid->dim != 0) return SR_E_UNSUPPORTED;      // uniform fields only
    if (prm->sampler == SR_SAMPLER_MLP || prm->omega_grid != 0.0) return SR_E_UNSUPPORTED;
    const sr_chunking chunks{(parts->n + kChunk - 1) / kChunk, nullptr};
    StepArgs<float> a;
    int64_t n_chunks = 0;
    const int rc = prepare_step<float>(parts, nullptr, grid, dt, seed, step0, prm, tab, &chunks,
                                       ph, led, false, a, n_chunks);
    if (rc != SR_OK) return rc;
    if (!led->rows || led->n_rows < n_steps) return SR_E_INVAL;
    if (led->partials_len < steps_partials(n_chunks, n_steps)) return SR_E_INVAL;
    if (n_chunks == 0) return SR_OK;
    hipStream_t st = (hipStream_t)stream;
    const int K = prm->n_samples;
    const int KM = K <= 1 ? 1 : K <= 2 ? 2 : K <= 4 ? 4 : K <= 8 ? 8 : 16;
    const unsigned nb = (unsigned)n_chunks;
#define SR_STEPS(KMV, SMP) push_emit_steps_kernel<KMV, SMP><<<nb, 64, 0, st>>>(a, n_steps)
#define SR_STEPS_K(SMP)                      \
    switch (KM) {                            \
        case 1: SR_STEPS(1, SMP); break;     \
        case 2: SR_STEPS(2, SMP); break;     \
        case 4: SR_STEPS(4, SMP); break;     \
        case 8: SR_STEPS(8, SMP); break;     \
        default: SR_STEPS(16, SMP); break;   \
    }
    if (prm->sampler == SR_SAMPLER_S) { SR_STEPS_K(SR_SAMPLER_S); }
    else if (prm->sampler == SR_SAMPLER_TABLE) { SR_STEPS_K(SR_SAMPLER_TABLE); }
    else { SR_STEPS_K(SR_SAMPLER_QUANTUM); }
#undef SR_STEPS_K
#undef SR_STEPS
    steps_reduce_kernel<<<(unsigned)n_steps, kBlock, 0, st>>>(led->partials, (int64_t)nb, led->rows,
                                                              led->status);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

// Gather, push and H_eff of every particle without emission or any write to
// the particles: out_heff, out_chi, out_gamma_bar (device FP64, n each).
template <typename R, int DIM>
__global__ __launch_bounds__(kBlock) void eval_push_kernel(const StepArgs<R> a,
                                                           double *__restrict__ heff,
                                                           double *__restrict__ chi,
                                                           double *__restrict__ gbar) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const uint32_t u = (uint32_t)i;
    R pos[3] = {(R)0, (R)0, (R)0};
    if (a.has_pos) {
        pos[0] = ld(a.x[0], u);
        if (DIM != 0 || a.x[1]) pos[1] = ld(a.x[1], u);
        if ((DIM == 3 || DIM == 0) && a.x[2]) pos[2] = ld(a.x[2], u);
    }
    const R p0[3] = {ld(a.p[0], u), ld(a.p[1], u), ld(a.p[2], u)};
    const Pushed<R> q = push_heff<R, DIM>(a, pos, p0);
    heff[i] = (double)q.H;
    chi[i] = (double)q.chi;
    gbar[i] = (double)q.gb;
}

// Validity diagnostics of the method's two stated limits, per particle (flag
// bits SR_VALID_*) and as weighted sums over the particles: {sum w, sum w
// [quantum], sum w [non-synchrotron], sum w LL, sum w LL [quantum], sum w LL
// [non-synchrotron]}, LL the Landau-Lifshitz energy of the step (the ledger's
// LL column).  Each block writes its sums to part[block][SR_VALID_SUMS]; a
// second kernel adds the blocks in a fixed order.
template <typename R, int DIM>
__global__ __launch_bounds__(kBlock) void validity_kernel(const StepArgs<R> a, R tau_em,
                                                          uint8_t *__restrict__ flags,
                                                          double *__restrict__ part) {
    __shared__ double sh[SR_VALID_SUMS][kWaves];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v[SR_VALID_SUMS];
#pragma unroll
    for (int c = 0; c < SR_VALID_SUMS; ++c) v[c] = 0.0;
    if (i < a.n) {
        const uint32_t u = (uint32_t)i;
        R pos[3] = {(R)0, (R)0, (R)0};
        if (a.has_pos) {
            pos[0] = ld(a.x[0], u);
            if (DIM != 0 || a.x[1]) pos[1] = ld(a.x[1], u);
            if ((DIM == 3 || DIM == 0) && a.x[2]) pos[2] = ld(a.x[2], u);
        }
        const R p0[3] = {ld(a.p[0], u), ld(a.p[1], u), ld(a.p[2], u)};
        const Pushed<R> q = push_heff<R, DIM>(a, pos, p0);
        const bool quantum = q.chi >= (R)1;
        const bool non_synch = q.H > (R)0 && q.H * tau_em <= (R)1;
        const uint32_t f = (quantum ? SR_VALID_QUANTUM : 0u) | (non_synch ? SR_VALID_NON_SYNCHROTRON : 0u);
        if (flags) st(flags, u, (uint8_t)f);
        const double w = (double)ld(a.w, u);
        const R beta2 = q.gb > (R)0 ? q.p2 * rcp_r<R>(q.gb * q.gb) : (R)0;
        const double ll = w * (double)(a.ll_c * q.chi * q.chi * beta2);
        v[0] = w;
        v[1] = quantum ? w : 0.0;
        v[2] = non_synch ? w : 0.0;
        v[3] = ll;
        v[4] = quantum ? ll : 0.0;
        v[5] = non_synch ? ll : 0.0;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < SR_VALID_SUMS; ++c) {
        const double t = wave_sum(v[c]);
        if (lane == 0) sh[c][wave] = t;
    }
    __syncthreads();
    if (threadIdx.x < SR_VALID_SUMS) {
        const int c = threadIdx.x;
        part[(int64_t)blockIdx.x * SR_VALID_SUMS + c] = ((sh[c][0] + sh[c][1]) + sh[c][2]) + sh[c][3];
    }
}

// out[c] = sum over the blocks of part[b][c], in block order within each thread's
// strided set, then a fixed tree over the threads.
__global__ __launch_bounds__(kBlock) void validity_reduce(const double *__restrict__ part,
                                                          int64_t n_blocks,
                                                          double *__restrict__ out) {
    __shared__ double sh[kWaves];
    const int c = blockIdx.x;
    double acc = 0.0;
    for (int64_t b = threadIdx.x; b < n_blocks; b += kBlock) acc += part[b * SR_VALID_SUMS + c];
    const double t = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) out[c] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

template <typename R, typename PARTS>
int launch_validity(PARTS *parts, const sr_fields_f32 *fields, const sr_grid *grid, double dt,
                    const sr_params *prm, double tau_em, uint8_t *flags, double *sums,
                    double *work, void *stream) {
    StepArgs<R> a;
    const int rc = particle_args<R>(parts, fields, grid, dt, prm, a);
    if (rc != SR_OK) return rc;
    if (!sums || !work || !(tau_em > 0.0) || !isfinite(tau_em)) return SR_E_INVAL;
    const int64_t nb = (parts->n + kBlock - 1) / kBlock;
    if (nb > 0x7fffffffLL) return SR_E_INVAL;
    hipStream_t st = (hipStream_t)stream;
    if (nb > 0) {
        switch (grid->dim) {
            case 0: validity_kernel<R, 0><<<(unsigned)nb, kBlock, 0, st>>>(a, (R)tau_em, flags, work); break;
            case 2: validity_kernel<R, 2><<<(unsigned)nb, kBlock, 0, st>>>(a, (R)tau_em, flags, work); break;
            default: validity_kernel<R, 3><<<(unsigned)nb, kBlock, 0, st>>>(a, (R)tau_em, flags, work); break;
        }
    }
    validity_reduce<<<SR_VALID_SUMS, kBlock, 0, st>>>(work, nb, sums);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

template <typename R, typename PARTS>
int launch_eval_push(PARTS *parts, const sr_fields_f32 *fields, const sr_grid *grid, double dt,
                     const sr_params *prm, double *heff, double *chi, double *gbar, void *stream) {
    StepArgs<R> a;
    const int rc = particle_args<R>(parts, fields, grid, dt, prm, a);
    if (rc != SR_OK) return rc;
    if (parts->n == 0) return SR_OK;
    if (!heff || !chi || !gbar) return SR_E_INVAL;
    const unsigned nb = (unsigned)((parts->n + kBlock - 1) / kBlock);
    hipStream_t st = (hipStream_t)stream;
    switch (grid->dim) {
        case 0: eval_push_kernel<R, 0><<<nb, kBlock, 0, st>>>(a, heff, chi, gbar); break;
        case 2: eval_push_kernel<R, 2><<<nb, kBlock, 0, st>>>(a, heff, chi, gbar); break;
        default: eval_push_kernel<R, 3><<<nb, kBlock, 0, st>>>(a, heff, chi, gbar); break;
    }
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the step that allocates nothing (sr_gather_push_emit_noalloc):
// the partial ledger rows of one step and the first level of their reduction,
// for up to kNoallocMaxChunks chunks, in one file-scope device array.  Each
// device holds its own copy at its own address; host code reaches it only
// through the address hipGetSymbolAddress gives on that device.
constexpr int64_t kNoallocMaxChunks = SR_NOALLOC_MAX_CHUNKS;
constexpr int64_t kNoallocDoubles =
    ((kNoallocMaxChunks + kWaves - 1) / kWaves + kReduceL1Blocks + 1) * kPartCols;
constexpr int kNoallocMaxDevices = 64;
static __device__ __align__(256) double scratch[kNoallocDoubles];

std::mutex g_scratch_mu;
double *g_scratch[kNoallocMaxDevices] = {};

// The device address of `scratch` on the current device, taken once per
// device (with that device current) and kept.
int scratch_on_current_device(double **out) {
    int dev = -1;
    SR_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoallocMaxDevices) return SR_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SR_E_HIP;
        g_scratch[dev] = (double *)ptr;
    }
    *out = g_scratch[dev];
    return SR_OK;
}

}  // namespace
}  // namespace sr

using namespace sr;

extern "C" int64_t sr_ledger_partials(int64_t n_chunks) {
    if (n_chunks < 0) return 0;
    return (partial_rows(n_chunks) + kReduceL1Blocks + 1) * kPartCols;
}

extern "C" int64_t sr_validity_work(int64_t n) {
    if (n < 0) return -1;
    return ((n + kBlock - 1) / kBlock) * SR_VALID_SUMS;
}

extern "C" int sr_validity(const sr_particles_f32 *parts, const sr_fields_f32 *fields,
                           const sr_grid *grid, double dt, const sr_params *prm, double tau_em,
                           uint8_t *flags, double *sums, double *work, void *stream) {
    return launch_validity<float>(parts, fields, grid, dt, prm, tau_em, flags, sums, work, stream);
}

extern "C" int sr_eval_push(const sr_particles_f32 *parts, const sr_fields_f32 *fields,
                            const sr_grid *grid, double dt, const sr_params *prm, double *out_heff,
                            double *out_chi, double *out_gamma_bar, void *stream) {
    return launch_eval_push<float>(parts, fields, grid, dt, prm, out_heff, out_chi, out_gamma_bar,
                                   stream);
}

extern "C" int sr_eval_push_f64(const sr_particles_f64 *parts, const sr_fields_f32 *fields,
                                const sr_grid *grid, double dt, const sr_params *prm,
                                double *out_heff, double *out_chi, double *out_gamma_bar,
                                void *stream) {
    return launch_eval_push<double>(parts, fields, grid, dt, prm, out_heff, out_chi,
                                    out_gamma_bar, stream);
}

extern "C" int sr_gather_push_emit(sr_particles_f32 *parts, const sr_fields_f32 *fields,
                                   const sr_grid *grid, double dt, uint64_t seed, uint64_t step,
                                   const sr_params *prm, const sr_table *tab,
                                   const sr_chunking *chunks, sr_photon_buf *photons,
                                   sr_ledger *ledger, void *stream) {
    return launch_step<float>(parts, fields, grid, dt, seed, step, prm, tab, chunks, photons,
                              ledger, stream);
}

extern "C" int sr_gather_push_emit_timed(sr_particles_f32 *parts, const sr_fields_f32 *fields,
                                         const sr_grid *grid, double dt, uint64_t seed,
                                         uint64_t step, const sr_params *prm, const sr_table *tab,
                                         const sr_chunking *chunks, sr_photon_buf *photons,
                                         sr_ledger *ledger, void *ev_start, void *ev_stop,
                                         void *stream) {
    return launch_step<float>(parts, fields, grid, dt, seed, step, prm, tab, chunks, photons,
                              ledger, stream, ev_start, ev_stop);
}

extern "C" int sr_gather_push_emit_f64(sr_particles_f64 *parts, const sr_fields_f32 *fields,
                                       const sr_grid *grid, double dt, uint64_t seed,
                                       uint64_t step, const sr_params *prm, const sr_table *tab,
                                       const sr_chunking *chunks, sr_photon_buf *photons,
                                       sr_ledger *ledger, void *stream) {
    return launch_step<double>(parts, fields, grid, dt, seed, step, prm, tab, chunks, photons,
                               ledger, stream);
}

extern "C" int sr_gather_push_emit_noalloc(sr_particles_f32 *parts, const sr_fields_f32 *fields,
                                           const sr_grid *grid, double dt, uint64_t seed,
                                           uint64_t step, const sr_params *prm,
                                           const sr_table *tab, const sr_chunking *chunks,
                                           sr_photon_buf *photons, double *ledger_row,
                                           uint32_t *status, void *stream) {
    if (!parts || !chunks || !ledger_row || !status || parts->n < 0) return SR_E_INVAL;
    const int64_t n_chunks =
        chunks->start ? chunks->n_chunks : (parts->n + kChunk - 1) / kChunk;
    if (n_chunks < 0) return SR_E_INVAL;
    if (n_chunks > kNoallocMaxChunks) return SR_E_UNSUPPORTED;
    // the scratch belongs to the current device; the stream must run there
    if (stream) {
        int cur = -1;
        hipDevice_t sdev = -1;
        SR_HIP_CHECK(hipGetDevice(&cur));
        SR_HIP_CHECK(hipStreamGetDevice((hipStream_t)stream, &sdev));
        if ((int)sdev != cur) return SR_E_INVAL;
    }
    double *ws = nullptr;
    const int rs = scratch_on_current_device(&ws);
    if (rs != SR_OK) return rs;
    sr_ledger led;
    led.rows = ledger_row;
    led.n_rows = 1;
    led.partials = ws;
    led.partials_len = kNoallocDoubles;
    led.status = status;
    const int rc = launch_step<float>(parts, fields, grid, dt, seed, step, prm, tab, chunks,
                                      photons, &led, stream);
    if (rc != SR_OK) return rc;
    return reduce_ledger(&led, n_chunks, 0, (hipStream_t)stream);
}

extern "C" int sr_gather_push_emit_steps(sr_particles_f32 *parts, const sr_grid *grid, double dt,
                                         uint64_t seed, uint64_t step0, int64_t n_steps,
                                         const sr_params *prm, const sr_table *tab,
                                         sr_photon_buf *photons, sr_ledger *ledger, void *stream) {
    return launch_steps(parts, grid, dt, seed, step0, n_steps, prm, tab, photons, ledger, stream);
}

extern "C" int64_t sr_ledger_partials_steps(int64_t n_chunks, int64_t n_steps) {
    if (n_chunks < 0 || n_steps < 0) return 0;
    return steps_partials(n_chunks, n_steps);
}

extern "C" int sr_ledger_reduce(const sr_ledger *ledger, int64_t n_chunks, int64_t row,
                                void *stream) {
    if (!ledger || !ledger->rows || !ledger->partials || !ledger->status || n_chunks < 0 ||
        n_chunks > 0x7FFFFFFF ||
        row < 0 || row >= ledger->n_rows || ledger->partials_len < sr_ledger_partials(n_chunks))
        return SR_E_INVAL;
    return reduce_ledger(ledger, n_chunks, row, (hipStream_t)stream);
}

extern "C" int sr_step_epilogue(const sr_ledger *ledger, int64_t n_chunks, int64_t row,
                                const sr_photon_buf *ph, const sr_chunking *chunks, int64_t n,
                                double eps_lo, double eps_hi, int32_t n_bins, double *hist,
                                double *work, void *stream) {
    // the argument checks of sr_ledger_reduce and of sr_spectrum_histogram
    if (!ledger || !ledger->rows || !ledger->partials || !ledger->status || n_chunks < 0 ||
        n_chunks > 0x7FFFFFFF ||
        row < 0 || row >= ledger->n_rows || ledger->partials_len < sr_ledger_partials(n_chunks))
        return SR_E_INVAL;
    if (!ph || !chunks || !hist || !work || n < 0 || n_bins < 1 || n_bins > kMaxBins ||
        !(eps_lo > 0.0) || !(eps_hi > eps_lo) || !ph->seg_count)
        return SR_E_INVAL;
    const int64_t h_chunks = chunks->start ? chunks->n_chunks : (n + kChunk - 1) / kChunk;
    const bool do_hist = h_chunks > 0 && ph->per_particle > 0;
    if (do_hist && (!ph->eps || !ph->w)) return SR_E_INVAL;
    const LedgerPlan lp = ledger_plan(ledger, n_chunks, row);
    const int nb_led = lp.mode == 2 ? (int)lp.nb : 1;
    const int nb_hist = do_hist ? hist_blocks(h_chunks) : 0;
    const float l2lo = (float)log2(eps_lo);
    const float scale = (float)(n_bins / (log2(eps_hi) - log2(eps_lo)));
    hipStream_t st = (hipStream_t)stream;
    epilogue_first_kernel<<<nb_led + nb_hist, kBlock, sizeof(double) * 2 * n_bins, st>>>(
        ledger->partials, lp.rows, lp.per, nb_led, lp.mode == 2 ? lp.mid : lp.dst,
        lp.mode == 2 ? nullptr : ledger->status, *ph, chunks->start, h_chunks, n, l2lo, scale,
        n_bins, work, nb_hist);
    const int led_blocks = lp.mode == 2 ? 1 : 0;
    const int second = led_blocks + (do_hist ? 2 * n_bins : 0);
    if (second > 0)
        epilogue_second_kernel<<<second, kBlock, 0, st>>>(lp.mid, lp.nb, lp.dst, ledger->status,
                                                          led_blocks, work, nb_hist, 2 * n_bins,
                                                          hist);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

extern "C" int sr_energy_ledger(const sr_ledger *led, int64_t row, double *out, void *stream) {
    if (!led || !out || !led->rows || row < 0 || row >= led->n_rows) return SR_E_INVAL;
    hipStream_t st = (hipStream_t)stream;
    SR_HIP_CHECK(hipMemcpyAsync(out, led->rows + row * SR_LEDGER_COLS,
                                sizeof(double) * SR_LEDGER_COLS, hipMemcpyDeviceToHost, st));
    SR_HIP_CHECK(hipStreamSynchronize(st));
    return SR_OK;
}

extern "C" int sr_status(const sr_ledger *led, uint32_t *flags, int32_t clear, void *stream) {
    if (!led || !flags || !led->status) return SR_E_INVAL;
    hipStream_t st = (hipStream_t)stream;
    SR_HIP_CHECK(hipMemcpyAsync(flags, led->status, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    if (clear) SR_HIP_CHECK(hipMemsetAsync(led->status, 0, sizeof(uint32_t), st));
    SR_HIP_CHECK(hipStreamSynchronize(st));
    return SR_OK;
}
