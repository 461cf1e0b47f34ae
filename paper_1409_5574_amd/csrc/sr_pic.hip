// sr_pic.hip -- closing the PIC loop around the emission step: the Yee field
// solve, the grid charge and the charge-conserving current of the particles'
// moves, and the ballistic motion of the emitted photons.
//
// The paper's emission method runs inside a PIC code: particles on a grid,
// Maxwell's equations for the field, the particles' currents feeding it
// (section "The field setup"); the photons it emits are particles that move at
// c along their direction.  Normalised units: E, B in m c omega_r / e, lengths
// in c/omega_r, densities in n_r = m omega_r^2 / (4 pi e^2), so
//     dB/dt = -curl E,   dE/dt = curl B - J,   div E = rho.
// A step keeps E and B at whole steps, where the particles gather them:
//     B -= (dt/2) curl E;   E += dt (curl B - J);   B -= (dt/2) curl E.
#include <math.h>

#include "sr_common.hpp"

namespace sr {
namespace {

// Grid geometry for the PIC kernels (positions from the lower corner).
struct PicGrid {
    int n[3];
    float inv_hi[3], inv_lo[3];   // 1/dx split so that x/dx keeps ~2^-24 absolute accuracy
    float L[3];                   // box lengths
    float dV;                     // cell volume (2D: dx dy)
};

inline int pic_grid(const sr_grid *g, PicGrid &G) {
    if (!g || (g->dim != 2 && g->dim != 3)) return SR_E_INVAL;
    if (g->dim == 2 && g->n[2] != 1) return SR_E_INVAL;
    int64_t cells = 1;
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 1 || g->n[a] > (1 << 24)) return SR_E_INVAL;
        if (a < g->dim && (!(g->dx[a] > 0.0) || !isfinite(g->dx[a]))) return SR_E_INVAL;
        cells *= g->n[a];
    }
    if (cells >= (int64_t)1 << 30) return SR_E_UNSUPPORTED;
    G.dV = 1.0f;
    for (int a = 0; a < 3; ++a) {
        G.n[a] = (int)g->n[a];
        const double inv = a < g->dim ? 1.0 / g->dx[a] : 0.0;
        G.inv_hi[a] = (float)inv;
        G.inv_lo[a] = (float)(inv - (double)G.inv_hi[a]);
        G.L[a] = a < g->dim ? (float)(g->n[a] * g->dx[a]) : 0.0f;
        if (a < g->dim) G.dV *= (float)g->dx[a];
    }
    return SR_OK;
}

__device__ __forceinline__ uint32_t cell(int i, int j, int k, const PicGrid &G) {
    return (uint32_t)i + (uint32_t)G.n[0] * ((uint32_t)j + (uint32_t)G.n[1] * (uint32_t)k);
}
__device__ __forceinline__ int up(int i, int n) { return i + 1 == n ? 0 : i + 1; }
__device__ __forceinline__ int dn(int i, int n) { return i == 0 ? n - 1 : i - 1; }

// ------------------------------------------------------------ Yee field solve
// B -= h curl E on the B points (forward differences), one thread per cell.
template <int DIM>
__global__ __launch_bounds__(256) void curl_e_kernel(const float *__restrict__ ex,
                                                     const float *__restrict__ ey,
                                                     const float *__restrict__ ez,
                                                     float *__restrict__ bx, float *__restrict__ by,
                                                     float *__restrict__ bz, PicGrid G, float hx,
                                                     float hy, float hz, uint32_t cells) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const int nx = G.n[0], ny = G.n[1];
    const int i = (int)(c % (uint32_t)nx), r = (int)(c / (uint32_t)nx);
    const int j = r % ny, k = r / ny;
    const uint32_t cx = cell(up(i, nx), j, k, G), cy = cell(i, up(j, ny), k, G);
    const float ex0 = ld(ex, c), ey0 = ld(ey, c), ez0 = ld(ez, c);
    // hx = h/dx etc.
    float dbx = hy * (ld(ez, cy) - ez0);
    float dby = -hx * (ld(ez, cx) - ez0);
    const float dbz = hx * (ld(ey, cx) - ey0) - hy * (ld(ex, cy) - ex0);
    if (DIM == 3) {
        const uint32_t cz = cell(i, j, up(k, G.n[2]), G);
        dbx -= hz * (ld(ey, cz) - ey0);
        dby += hz * (ld(ex, cz) - ex0);
    }
    st(bx, c, ld(bx, c) - dbx);
    st(by, c, ld(by, c) - dby);
    st(bz, c, ld(bz, c) - dbz);
}

// E += dt (curl B - J) on the E points (backward differences).
template <int DIM, bool HAS_J>
__global__ __launch_bounds__(256) void curl_b_kernel(float *__restrict__ ex, float *__restrict__ ey,
                                                     float *__restrict__ ez,
                                                     const float *__restrict__ bx,
                                                     const float *__restrict__ by,
                                                     const float *__restrict__ bz,
                                                     const float *__restrict__ jx,
                                                     const float *__restrict__ jy,
                                                     const float *__restrict__ jz, PicGrid G,
                                                     float dt, float tx, float ty, float tz,
                                                     uint32_t cells) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const int nx = G.n[0], ny = G.n[1];
    const int i = (int)(c % (uint32_t)nx), r = (int)(c / (uint32_t)nx);
    const int j = r % ny, k = r / ny;
    const uint32_t cx = cell(dn(i, nx), j, k, G), cy = cell(i, dn(j, ny), k, G);
    const float bx0 = ld(bx, c), by0 = ld(by, c), bz0 = ld(bz, c);
    // tx = dt/dx etc.
    float dex = ty * (bz0 - ld(bz, cy));
    float dey = -tx * (bz0 - ld(bz, cx));
    float dez = tx * (by0 - ld(by, cx)) - ty * (bx0 - ld(bx, cy));
    if (DIM == 3) {
        const uint32_t cz = cell(i, j, dn(k, G.n[2]), G);
        dex -= tz * (by0 - ld(by, cz));
        dey += tz * (bx0 - ld(bx, cz));
    }
    if (HAS_J) {
        dex = fmaf(-dt, ld(jx, c), dex);
        dey = fmaf(-dt, ld(jy, c), dey);
        dez = fmaf(-dt, ld(jz, c), dez);
    }
    st(ex, c, ld(ex, c) + dex);
    st(ey, c, ld(ey, c) + dey);
    st(ez, c, ld(ez, c) + dez);
}

// --------------------------------------------------- charge and current
// Position on one axis as (cell index, fraction in [0, 1)).
__device__ __forceinline__ void locate(float x, float inv_hi, float inv_lo, int n, int &i, float &f) {
    const float u = x * inv_hi;
    float fi = floorf(u);
    float fr = fmaf(x, inv_hi, -fi) + x * inv_lo;
    if (fr < 0.0f) { fr += 1.0f; fi -= 1.0f; }
    if (fr >= 1.0f) { fr -= 1.0f; fi += 1.0f; }
    i = (int)fi;
    i = i < 0 ? i + n : (i >= n ? i - n : i);
    i = min(max(i, 0), n - 1);
    f = fr;
}

// Node index base + c (c = 0..3, base = i - 1) wrapped into [0, n).
__device__ __forceinline__ int node(int i, int c, int n) {
    int v = i - 1 + c;
    v = v < 0 ? v + n : (v >= n ? v - n : v);
    return min(max(v, 0), n - 1);
}

// l / d for 0 <= l < 2^22 and d >= 1, from a float reciprocal: the product
// is within one of the quotient, and one step each way corrects it
__device__ __forceinline__ int div_small(int l, int d, float inv_d) {
    int q = (int)((float)l * inv_d);
    q -= q * d > l ? 1 : 0;
    q += (q + 1) * d <= l ? 1 : 0;
    return q;
}

// i in [-2n, 3n) onto [0, n)
__device__ __forceinline__ int wrap2(int i, int n) {
    if (i < 0) i += n;
    if (i < 0) i += n;
    if (i >= n) i -= n;
    if (i >= n) i -= n;
    return i;
}

// CIC weight of a particle at relative coordinate r (cells from node i) on the
// node i - 1 + c.
__device__ __forceinline__ float cic_w(float r, int c) {
    return fmaxf(0.0f, 1.0f - fabsf(r - (float)(c - 1)));
}

// Charge: rho += q w S / dV on the 4 (2D) or 8 (3D) nodes of each particle.
template <int DIM>
__global__ __launch_bounds__(256) void rho_kernel(sr_particles_f32 P, PicGrid G, float qv,
                                                  float *__restrict__ rho) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n) return;
    const uint32_t u = (uint32_t)p;
    int I[3] = {0, 0, 0};
    float F[3] = {0.0f, 0.0f, 0.0f};
    for (int a = 0; a < DIM; ++a) locate(ld(P.x[a], u), G.inv_hi[a], G.inv_lo[a], G.n[a], I[a], F[a]);
    const float qw = qv * ld(P.w, u) / G.dV;
    for (int c = 0; c < (DIM == 3 ? 2 : 1); ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const float wt = (a ? F[0] : 1.0f - F[0]) * (b ? F[1] : 1.0f - F[1]) *
                                 (DIM == 3 ? (c ? F[2] : 1.0f - F[2]) : 1.0f);
                const int i = node(I[0], 1 + a, G.n[0]), j = node(I[1], 1 + b, G.n[1]);
                const int k = DIM == 3 ? node(I[2], 1 + c, G.n[2]) : 0;
                unsafeAtomicAdd(&rho[cell(i, j, k, G)], qw * wt);
            }
}

// Esirkepov's current of the move x_old -> x (one lane per particle).  On each
// axis the old shape S0 and the new shape S1 of a move below one cell lie on
// three consecutive nodes among i-1 .. i+2 of the old cell i, and the loops
// run over those three; D = S1 - S0.  Per node of the stencil
//   3D  W_x = Dx (S0y S0z + Dy S0z/2 + S0y Dz/2 + Dy Dz/3)  (and cyclically),
//   Jx(i+1/2) = Jx(i-1/2) - q w (dx/dt) W_x / dV, summed along x;
//   2D  W_x = Dx (S0y + Dy/2),  W_y = Dy (S0x + Dx/2),
//       Jz = q w v_z (S0x S0y + Dx S0y/2 + S0x Dy/2 + Dx Dy/3) / dV on the nodes.
// Zero contributions are skipped.  A move of a cell or more sets *status.
//
// Sorted particles put the lanes of a block on the same few cells, where
// global float atomics serialise.  So the block first finds the box of nodes
// its particles touch, with cells taken relative to the block's first particle
// across the periodic boundary (a block whose sorted particles run from the end
// of one tile row into the next keeps a compact box).  If that box fits in LDS
// (kDepCells cells, three components) the block accumulates there and adds the
// box's non-zero entries to the grid at the end.  A larger box (particles that
// have drifted far since the last sort) shrinks to a window of at most
// kDepCells cells about the block's mean cell, and only the particles whose
// nodes leave the window add to the grid directly.
//
// The box holds fixed-point integers, not floats: on gfx950 an LDS float
// atomic add takes about 40 times as long as an integer one, and it was the
// bulk of the deposit's time.  Each contribution v is rounded to an integer
// multiple of 2^(e-21), where 2^e bounds every contribution of the block: on
// each axis |v| <= |c_a| |du_a| (the partial sums of D over a hat shape are
// bounded by the move du in cells, the transverse factor lies in [0, 1]), and
// |v| <= |c_z| for the 2D Jz.  A node takes at most one contribution per
// particle and component, so a sum stays below 512 * 2^21 = 2^30, and the
// integer adds are exact and independent of order.  The rounding error per
// contribution is at most half a unit, 2^(e-22) <= 2^-21 B with B the block's
// largest bound, so a node's block sum is within n 2^-21 B <= 2^-12 B of the
// exact sum of its n <= 512 contributions.  That bound is absolute: a node
// whose current is far below B in a block that also holds a much heavier or
// faster particle keeps only that absolute accuracy.
constexpr int kDepThreads = 512;   // particles per block
constexpr int kDepWaves = kDepThreads / 64;
constexpr int kDepCells = 3072;
// 2^kDepFracBits units per bound and at most kDepThreads contributions per
// node: sums stay below 2^30
constexpr int kDepFracBits = 30 - 9;
static_assert(kDepThreads == 512, "kDepFracBits assumes 2^9 particles per block");

struct Stencil {
    int I[3];              // old cell of the particle on each axis
    int o[3];              // the move's three nodes on each axis: I - 1 + o .. I + 1 + o
    float S0[3][3], D[3][3];   // old shape and its change on those nodes
    float cx, cy, cz;      // -q w (dx_a/dt)/dV (3D), and q w v_z / dV for 2D Jz in cz
    float bound;           // bound on |contribution| (with a margin for rounding)
    bool live;             // active, finite move below one cell
};

template <int DIM>
__device__ __forceinline__ Stencil make_stencil(const sr_particles_f32 &P, const float *const xo[3],
                                                const PicGrid &G, float qv, float inv_dt,
                                                uint32_t u, bool active, bool &bad) {
    Stencil s;
    s.live = active;
    bad = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s.I[a] = 0;
        s.o[a] = 1;
        for (int c = 0; c < 3; ++c) { s.S0[a][c] = (a >= DIM && c == 0) ? 1.0f : 0.0f; s.D[a][c] = 0.0f; }
    }
    s.cx = s.cy = s.cz = 0.0f;
    s.bound = 0.0f;
    if (!active) return s;
    bool ok = true;
    float du_abs[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const float x0 = ld(xo[a], u), x1 = ld(P.x[a], u);
        float d = x1 - x0;                       // the shorter way round the box
        if (d > 0.5f * G.L[a]) d -= G.L[a];
        else if (d < -0.5f * G.L[a]) d += G.L[a];
        float f0;
        locate(x0, G.inv_hi[a], G.inv_lo[a], G.n[a], s.I[a], f0);
        const float du = d * G.inv_hi[a];
        ok = ok && fabsf(du) < 1.0f;
        du_abs[a] = fabsf(du);
        const float r1 = f0 + du;
        // old shape on nodes i, i+1; new shape on i-1, i (r1 < 0) or on
        // i, i+1 or i+1, i+2: three nodes from i - 1 + o
        const int o = r1 < 0.0f ? 0 : 1;
        s.o[a] = o;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            s.S0[a][c] = cic_w(f0, c + o);
            s.D[a][c] = cic_w(r1, c + o) - s.S0[a][c];
        }
    }
    if (!ok) {
        bad = true;
        s.live = false;
        return s;
    }
    const float qw = qv * ld(P.w, u);
    const float inv_dV = 1.0f / G.dV;
    s.cx = -qw * inv_dt * inv_dV / (G.inv_hi[0] + G.inv_lo[0]);
    s.cy = -qw * inv_dt * inv_dV / (G.inv_hi[1] + G.inv_lo[1]);
    if (DIM == 3) {
        s.cz = -qw * inv_dt * inv_dV / (G.inv_hi[2] + G.inv_lo[2]);
    } else {
        // v_z of the move from the momentum the position push used
        const float pz = ld(P.p[2], u), px = ld(P.p[0], u), py = ld(P.p[1], u);
        s.cz = qw * pz * __builtin_amdgcn_rsqf(1.0f + px * px + py * py + pz * pz) * inv_dV;
    }
    // |v| <= |c_a| |du_a| per axis (2D Jz: |c_z|); the margin covers the
    // rounding of the weights and of their partial sums
    constexpr float kPad = 1.0f / (1 << 20);
    float b = fmaxf(fabsf(s.cx) * (du_abs[0] + kPad), fabsf(s.cy) * (du_abs[1] + kPad));
    b = fmaxf(b, DIM == 3 ? fabsf(s.cz) * (du_abs[2] + kPad) : fabsf(s.cz));
    s.bound = b * 1.001f;
    return s;
}

// Every non-zero contribution of one particle, as add(component, node offsets
// ci, cj, ck in 0..2 relative to I - 1 + o, value).  Along the component's own
// axis only the first two partial sums are stored: the third is the sum of D,
// which is zero.
template <int DIM, typename ADD>
__device__ __forceinline__ void esirkepov(const Stencil &s, ADD &&add) {
    if (DIM == 3) {
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 3; ++j) {
                const float f = s.S0[1][j] * s.S0[2][k] + 0.5f * s.D[1][j] * s.S0[2][k] +
                                0.5f * s.S0[1][j] * s.D[2][k] + s.D[1][j] * s.D[2][k] * (1.0f / 3.0f);
                if (f == 0.0f) continue;
                float acc = 0.0f;
                for (int i = 0; i < 2; ++i) {
                    acc += s.cx * s.D[0][i] * f;
                    if (acc != 0.0f) add(0, i, j, k, acc);
                }
            }
        for (int k = 0; k < 3; ++k)
            for (int i = 0; i < 3; ++i) {
                const float f = s.S0[0][i] * s.S0[2][k] + 0.5f * s.D[0][i] * s.S0[2][k] +
                                0.5f * s.S0[0][i] * s.D[2][k] + s.D[0][i] * s.D[2][k] * (1.0f / 3.0f);
                if (f == 0.0f) continue;
                float acc = 0.0f;
                for (int j = 0; j < 2; ++j) {
                    acc += s.cy * s.D[1][j] * f;
                    if (acc != 0.0f) add(1, i, j, k, acc);
                }
            }
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) {
                const float f = s.S0[0][i] * s.S0[1][j] + 0.5f * s.D[0][i] * s.S0[1][j] +
                                0.5f * s.S0[0][i] * s.D[1][j] + s.D[0][i] * s.D[1][j] * (1.0f / 3.0f);
                if (f == 0.0f) continue;
                float acc = 0.0f;
                for (int k = 0; k < 2; ++k) {
                    acc += s.cz * s.D[2][k] * f;
                    if (acc != 0.0f) add(2, i, j, k, acc);
                }
            }
    } else {
        for (int j = 0; j < 3; ++j) {
            const float f = s.S0[1][j] + 0.5f * s.D[1][j];
            if (f == 0.0f) continue;
            float acc = 0.0f;
            for (int i = 0; i < 2; ++i) {
                acc += s.cx * s.D[0][i] * f;
                if (acc != 0.0f) add(0, i, j, 0, acc);
            }
        }
        for (int i = 0; i < 3; ++i) {
            const float f = s.S0[0][i] + 0.5f * s.D[0][i];
            if (f == 0.0f) continue;
            float acc = 0.0f;
            for (int j = 0; j < 2; ++j) {
                acc += s.cy * s.D[1][j] * f;
                if (acc != 0.0f) add(1, i, j, 0, acc);
            }
        }
        if (s.cz != 0.0f)
            for (int j = 0; j < 3; ++j)
                for (int i = 0; i < 3; ++i) {
                    const float wt = s.S0[0][i] * s.S0[1][j] + 0.5f * s.D[0][i] * s.S0[1][j] +
                                     0.5f * s.S0[0][i] * s.D[1][j] + s.D[0][i] * s.D[1][j] * (1.0f / 3.0f);
                    if (wt != 0.0f) add(2, i, j, 0, s.cz * wt);
                }
    }
}

template <int DIM>
__global__ __launch_bounds__(kDepThreads) void current_kernel(sr_particles_f32 P, const float *xo0,
                                                      const float *xo1, const float *xo2,
                                                      PicGrid G, float qv, float inv_dt,
                                                      float *__restrict__ jx, float *__restrict__ jy,
                                                      float *__restrict__ jz,
                                                      uint32_t *__restrict__ status) {
    __shared__ int box[3 * kDepCells];
    __shared__ int red[2][3][kDepWaves];
    __shared__ float bmax[kDepWaves];
    __shared__ int ref[3];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = p < P.n;
    const uint32_t u = active ? (uint32_t)p : 0u;
    const float *const xo[3] = {xo0, xo1, xo2};
    bool bad;
    const Stencil s = make_stencil<DIM>(P, xo, G, qv, inv_dt, u, active, bad);
    if (bad) atomicOr(status, SR_W_CFL);
    float *const J[3] = {jx, jy, jz};

    // the cells relative to the block's first particle (always active: the
    // grid has ceil(n / kDepThreads) blocks), unwrapped across the periodic boundary
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) ref[a] = s.I[a];
    __syncthreads();
    int U[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int d = s.I[a] - ref[a];
        if (a < DIM) {
            if (2 * d > G.n[a]) d -= G.n[a];
            else if (2 * d < -G.n[a]) d += G.n[a];
        }
        U[a] = ref[a] + d;
    }

    // the block's box of nodes [min U - 1, max U + 2] and its largest bound
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int lo = s.live ? U[a] : 0x3fffffff, hi = s.live ? U[a] : -0x3fffffff;
        for (int o = 32; o > 0; o >>= 1) {
            lo = min(lo, __shfl_xor(lo, o, 64));
            hi = max(hi, __shfl_xor(hi, o, 64));
        }
        if (lane == 0) { red[0][a][wave] = lo; red[1][a][wave] = hi; }
    }
    {
        // a non-finite bound (a NaN or infinite weight) counts as infinite
        float b = s.live ? (s.bound <= 3.0e38f ? s.bound : __builtin_inff()) : 0.0f;
        for (int o = 32; o > 0; o >>= 1) b = fmaxf(b, __shfl_xor(b, o, 64));
        if (lane == 0) bmax[wave] = b;
    }
    __syncthreads();
    int org[3], ext[3];
    bool any = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int lo = red[0][a][0], hi = red[1][a][0];
        for (int w = 1; w < kDepWaves; ++w) { lo = min(lo, red[0][a][w]); hi = max(hi, red[1][a][w]); }
        any = any && hi >= lo;      // no live particle: lo > hi
        if (a < DIM) {
            org[a] = lo - 1;
            ext[a] = hi - lo + 4;
        } else {
            org[a] = 0;
            ext[a] = 1;
        }
    }
    if (!any) return;               // no live particle (the condition is block-wide)
    float bnd = bmax[0];
    for (int w = 1; w < kDepWaves; ++w) bnd = fmaxf(bnd, bmax[w]);
    // bnd < 2^e: contributions in units of 2^(e - kDepFracBits).  A
    // non-finite bound, or one so small that 2^(kDepFracBits - e) would not
    // be a finite float, sends the whole block to the float path.
    int e = 0;
    if (bnd > 0.0f) (void)frexpf(bnd, &e);
    const bool fixed = bnd <= 3.0e38f && e >= -100;
    // A box too large for LDS shrinks, widest axis first, to a window about
    // the block's mean cell (kept inside the box); the particles whose nodes
    // leave the window add to the grid directly.  Volumes in 64 bits: extents
    // can be as large as the grid.
    int64_t vol = (int64_t)ext[0] * ext[1] * ext[2];
    if (fixed && vol > kDepCells) {
        __shared__ float msum[3][kDepWaves];
        __shared__ int mcnt[kDepWaves];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float v = s.live ? (float)(U[a] - ref[a]) : 0.0f;
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) msum[a][wave] = v;
        }
        int live = s.live ? 1 : 0;
        for (int o = 32; o > 0; o >>= 1) live += __shfl_xor(live, o, 64);
        if (lane == 0) mcnt[wave] = live;
        __syncthreads();
        int cnt = 0;
        for (int w = 0; w < kDepWaves; ++w) cnt += mcnt[w];
        for (int it = 0; it < DIM && vol > kDepCells; ++it) {
            int a = 0;
            for (int b = 1; b < DIM; ++b)
                if (ext[b] > ext[a]) a = b;
            const int64_t other = vol / ext[a];
            const int wdt = (int)min<int64_t>(ext[a], max<int64_t>(4, kDepCells / other));
            float sum = 0.0f;
            for (int w = 0; w < kDepWaves; ++w) sum += msum[a][w];
            const int c = ref[a] + (int)floorf(sum / (float)max(cnt, 1) + 0.5f);
            org[a] = min(max(c - wdt / 2, org[a]), org[a] + ext[a] - wdt);
            ext[a] = wdt;
            vol = other * wdt;
        }
    }
    bool in_win = s.live && fixed;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int b = U[a] - 1 + s.o[a] - org[a];
        in_win = in_win && b >= 0 && b + 2 <= ext[a] - 1;
    }
    if (s.live && !in_win)
        esirkepov<DIM>(s, [&](int comp, int ci, int cj, int ck, float v) {
            const int i = node(s.I[0], s.o[0] + ci, G.n[0]), j = node(s.I[1], s.o[1] + cj, G.n[1]);
            const int k = DIM == 3 ? node(s.I[2], s.o[2] + ck, G.n[2]) : 0;
            unsafeAtomicAdd(&J[comp][cell(i, j, k, G)], v);
        });
    if (!fixed || !(bnd > 0.0f)) return;      // block-wide; bnd = 0: every contribution is zero
    const float to_fix = ldexpf(1.0f, kDepFracBits - e), from_fix = ldexpf(1.0f, e - kDepFracBits);
    const int cells = ext[0] * ext[1] * ext[2];
    for (int q = threadIdx.x; q < 3 * cells; q += blockDim.x) box[q] = 0;
    __syncthreads();
    if (in_win) {
        const int b0 = U[0] - 1 + s.o[0] - org[0], b1 = U[1] - 1 + s.o[1] - org[1];
        const int b2 = DIM == 3 ? U[2] - 1 + s.o[2] - org[2] : 0;
        esirkepov<DIM>(s, [&](int comp, int ci, int cj, int ck, float v) {
            const int l = (b0 + ci) + ext[0] * ((b1 + cj) + ext[1] * (b2 + ck));
            atomicAdd(&box[comp * cells + l], __float2int_rn(v * to_fix));
        });
    }
    __syncthreads();
    const float inv_cells = 1.0f / (float)cells, inv_e0 = 1.0f / (float)ext[0];
    const float inv_e1 = 1.0f / (float)ext[1];
    for (int q = threadIdx.x; q < 3 * cells; q += blockDim.x) {
        const int sum = box[q];
        if (sum == 0) continue;
        const int comp = div_small(q, cells, inv_cells), l = q - comp * cells;
        const int r = div_small(l, ext[0], inv_e0), li = l - r * ext[0];
        const int lk = div_small(r, ext[1], inv_e1), lj = r - lk * ext[1];
        // the box's nodes wrapped onto the periodic grid: they lie in
        // [-n/2 - 1, 3n/2 + 1], so two wraps each way reach [0, n) for any n
        int i = org[0] + li, j = org[1] + lj, k = org[2] + lk;
        i = wrap2(i, G.n[0]);
        j = wrap2(j, G.n[1]);
        k = DIM == 3 ? wrap2(k, G.n[2]) : 0;
        i = min(max(i, 0), G.n[0] - 1);
        j = min(max(j, 0), G.n[1] - 1);
        k = min(max(k, 0), G.n[2] - 1);
        unsafeAtomicAdd(&J[comp][cell(i, j, k, G)], (float)sum * from_fix);
    }
}

// Photons move at c along their direction: pos += dt dir, wrapped into the box
// (one lane per chunk segment, as the photon histograms).
__global__ __launch_bounds__(256) void photon_advance_kernel(sr_photon_buf ph, const int64_t *start,
                                                             int64_t n_chunks, int64_t n, PicGrid G,
                                                             int dim, float dt) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_chunks) return;
    const int64_t s0 = start ? start[c] : c * (int64_t)kChunk;
    const int64_t e0 = start ? start[c + 1] : min(s0 + (int64_t)kChunk, n);
    const int64_t cap = (e0 - s0) * ph.per_particle;
    const int64_t cnt = min((int64_t)ph.seg_count[c], cap);
    const int64_t base = s0 * ph.per_particle;
    for (int64_t q = 0; q < cnt; ++q) {
        const uint32_t o = (uint32_t)(base + q);
        for (int a = 0; a < 3; ++a) {
            if (!ph.pos[a]) continue;
            float v = fmaf(dt, ld(ph.dir[a], o), ld(ph.pos[a], o));
            if (a < dim) {
                const float L = G.L[a];
                v -= L * floorf(v / L);
                if (v >= L || v < 0.0f) v = 0.0f;   // rounding guard (and a corrupt value)
            }
            st(ph.pos[a], o, v);
        }
    }
}

}  // namespace
}  // namespace sr

using namespace sr;

extern "C" int sr_field_step(float *e[3], float *b[3], const float *j[3], const sr_grid *grid,
                             double dt, void *stream) {
    PicGrid G;
    const int rc = pic_grid(grid, G);
    if (rc != SR_OK) return rc;
    if (!e || !b) return SR_E_INVAL;
    for (int q = 0; q < 3; ++q)
        if (!e[q] || !b[q]) return SR_E_INVAL;
    const bool has_j = j && j[0];
    if (has_j && (!j[1] || !j[2])) return SR_E_INVAL;
    // Courant condition of the Yee scheme: dt^2 (sum 1/dx_a^2) < 1
    double s = 0.0;
    for (int a = 0; a < grid->dim; ++a) s += 1.0 / (grid->dx[a] * grid->dx[a]);
    if (!(dt > 0.0) || !(dt * dt * s < 1.0)) return SR_E_INVAL;
    const uint32_t cells = (uint32_t)(grid->n[0] * grid->n[1] * grid->n[2]);
    const unsigned nb = (cells + 255) / 256;
    hipStream_t st = (hipStream_t)stream;
    const float h[3] = {(float)(0.5 * dt / grid->dx[0]), (float)(0.5 * dt / grid->dx[1]),
                        grid->dim == 3 ? (float)(0.5 * dt / grid->dx[2]) : 0.0f};
    const float t[3] = {2.0f * h[0], 2.0f * h[1], 2.0f * h[2]};
    for (int half = 0; half < 3; ++half) {
        if (half == 1) {
            if (grid->dim == 3) {
                if (has_j) curl_b_kernel<3, true><<<nb, 256, 0, st>>>(e[0], e[1], e[2], b[0], b[1], b[2], j[0], j[1], j[2], G, (float)dt, t[0], t[1], t[2], cells);
                else curl_b_kernel<3, false><<<nb, 256, 0, st>>>(e[0], e[1], e[2], b[0], b[1], b[2], nullptr, nullptr, nullptr, G, (float)dt, t[0], t[1], t[2], cells);
            } else {
                if (has_j) curl_b_kernel<2, true><<<nb, 256, 0, st>>>(e[0], e[1], e[2], b[0], b[1], b[2], j[0], j[1], j[2], G, (float)dt, t[0], t[1], t[2], cells);
                else curl_b_kernel<2, false><<<nb, 256, 0, st>>>(e[0], e[1], e[2], b[0], b[1], b[2], nullptr, nullptr, nullptr, G, (float)dt, t[0], t[1], t[2], cells);
            }
        } else {
            if (grid->dim == 3)
                curl_e_kernel<3><<<nb, 256, 0, st>>>(e[0], e[1], e[2], b[0], b[1], b[2], G, h[0], h[1], h[2], cells);
            else
                curl_e_kernel<2><<<nb, 256, 0, st>>>(e[0], e[1], e[2], b[0], b[1], b[2], G, h[0], h[1], h[2], cells);
        }
    }
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

extern "C" int sr_deposit_rho(const sr_particles_f32 *parts, const sr_grid *grid, double charge,
                              float *rho, void *stream) {
    PicGrid G;
    const int rc = pic_grid(grid, G);
    if (rc != SR_OK) return rc;
    if (!parts || !rho || parts->n < 0) return SR_E_INVAL;
    // element offsets are formed as 32-bit byte offsets (below 2^31 bytes)
    if (parts->n >= ((int64_t)1 << 29)) return SR_E_UNSUPPORTED;
    if (parts->n == 0) return SR_OK;
    if (!parts->x[0] || !parts->x[1] || (grid->dim == 3 && !parts->x[2]) || !parts->w)
        return SR_E_INVAL;
    const unsigned nb = (unsigned)((parts->n + 255) / 256);
    hipStream_t st = (hipStream_t)stream;
    if (grid->dim == 3) rho_kernel<3><<<nb, 256, 0, st>>>(*parts, G, (float)charge, rho);
    else rho_kernel<2><<<nb, 256, 0, st>>>(*parts, G, (float)charge, rho);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

extern "C" int sr_deposit_current(const sr_particles_f32 *parts, const float *x_old[3],
                                  const sr_grid *grid, double dt, double charge, float *j[3],
                                  uint32_t *status, void *stream) {
    PicGrid G;
    const int rc = pic_grid(grid, G);
    if (rc != SR_OK) return rc;
    if (!parts || !x_old || !j || !status || !(dt > 0.0) || parts->n < 0) return SR_E_INVAL;
    // element offsets are formed as 32-bit byte offsets (below 2^31 bytes)
    if (parts->n >= ((int64_t)1 << 29)) return SR_E_UNSUPPORTED;
    for (int q = 0; q < 3; ++q)
        if (!j[q]) return SR_E_INVAL;
    if (parts->n == 0) return SR_OK;
    const int dim = grid->dim;
    for (int a = 0; a < dim; ++a)
        if (!parts->x[a] || !x_old[a]) return SR_E_INVAL;
    if (!parts->w || (dim == 2 && (!parts->p[0] || !parts->p[1] || !parts->p[2])))
        return SR_E_INVAL;
    const unsigned nb = (unsigned)((parts->n + kDepThreads - 1) / kDepThreads);
    hipStream_t st = (hipStream_t)stream;
    if (dim == 3)
        current_kernel<3><<<nb, kDepThreads, 0, st>>>(*parts, x_old[0], x_old[1], x_old[2], G, (float)charge,
                                              (float)(1.0 / dt), j[0], j[1], j[2], status);
    else
        current_kernel<2><<<nb, kDepThreads, 0, st>>>(*parts, x_old[0], x_old[1], nullptr, G, (float)charge,
                                              (float)(1.0 / dt), j[0], j[1], j[2], status);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

extern "C" int sr_photon_advance(const sr_photon_buf *ph, const sr_chunking *chunks, int64_t n,
                                 const sr_grid *grid, double dt, void *stream) {
    PicGrid G;
    const int rc = pic_grid(grid, G);
    if (rc != SR_OK) return rc;
    if (!ph || !chunks || n < 0 || !ph->seg_count || !(dt >= 0.0)) return SR_E_INVAL;
    const int64_t n_chunks = chunks->start ? chunks->n_chunks : (n + kChunk - 1) / kChunk;
    if (n_chunks == 0 || ph->per_particle == 0) return SR_OK;
    if (!ph->dir[0] || !ph->dir[1] || !ph->dir[2]) return SR_E_INVAL;
    // photon slots are addressed with 32-bit byte offsets (below 2^32 bytes)
    if (n * ph->per_particle >= ((int64_t)1 << 30)) return SR_E_UNSUPPORTED;
    const unsigned nb = (unsigned)((n_chunks + 255) / 256);
    photon_advance_kernel<<<nb, 256, 0, (hipStream_t)stream>>>(*ph, chunks->start, n_chunks, n, G,
                                                               grid->dim, (float)dt);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}
