// spgm.hip -- gfx950 kernels and C-ABI of the matrix-free SPGM near-field MIMO projector.
//
// The observation matrix of Sec. II, Eq. 2,
//     A_{m,n} = p(f_m) exp(-j 2 pi f_m (d_T + d_R) / c) / (4 pi d_T d_R),
// is never stored: every launch forms the entries of its (row chunk x voxel tile) block in
// registers and applies them at once.  One SPGM iteration (Sec. IV, Eq. 5 with the gradient of
// Eq. 6) is five launches on the caller's stream:
//   1. k_sort_rows   sort the minibatch by (G antenna, L antenna, frequency) so that rows that
//                    share an antenna pair are adjacent and share their per-voxel geometry;
//   2. k_fwd_tile    per (voxel brick, row range): partial row sums of A_B s over the brick;
//   3. k_row_reduce  per row: sum of the brick partials in a fixed order, times p(f)/(4 pi),
//                    minus y_m (the residual of Eq. 6), pre-multiplied by conj(p(f)/(4 pi));
//   4. k_adj_tile    per (voxel brick, row range): partial column sums of A_B^H r, one voxel
//                    per lane and no atomics;
//   5. k_col_reduce  per voxel: sum of the row-range partials in a fixed order, gradient step
//                    and complex soft threshold (the prox of the l1 norm in Eq. 5).
// Every reduction runs in a fixed order, so results are bitwise reproducible run to run.
//
// Geometry per tile.  The grid is cut into 8 x 8 x 4 voxel bricks, one brick per work-group.
// Each of the work-group's eight waves covers the whole brick (a lane owns one (x, y) column
// of 4 voxels) and takes its own share of the rows, so the brick's LDS tables are shared by
// eight waves.  The two antenna arrays are called
// G (the sort-major side, whose per-voxel distance terms live in registers and are rebuilt when
// the G antenna changes) and L (the other side, whose per-voxel terms are staged in LDS for
// every L antenna).  L is the smaller array.
//
// Phase (SPGM_PHASE_COMP32).  With c the brick centre, e = r_n - c and g_a = c - r_a,
//     d_{a,n} - d_{a,c} = (|e|^2 + 2 e.g_a) / (d_{a,n} + d_{a,c})
// holds exactly and is evaluated in float32 with small relative error because |e| is a few
// millimetres.  The round-trip phase in turns is split as
//     f/c (d_T + d_R) = [f/c (d_{T,c} + d_{R,c})  mod 1]  +  f/c (delta_T + delta_R),
// the first term formed in float64 once per (row, brick), the second in float32 per entry.
// The result lies within a few turns of zero, where v_sin_f32 / v_cos_f32 (argument in turns)
// are accurate to about 1.2e-7 absolute, so no further range reduction is applied.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "spgm.h"

// Workspace of spgm_step_noalloc: a fixed device array, one copy on every GPU the library runs
// on, held until the process ends.  Host code never passes this name to a kernel (on the host
// it is only a stand-in for the symbol); it uses the device address resolved per device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kWave = 64;
constexpr int kWaves = 8;                     // waves per work-group, all on the same brick
constexpr int kThreads = kWaves * 64;
constexpr int kBX = 8, kBY = 8, kBZ = 4;      // voxel brick
constexpr int kBrick = kBX * kBY * kBZ;       // 256 voxels, one (x, y) column per lane
constexpr int kP = kBZ;                       // voxels per lane
constexpr int kSub = kThreads;                // rows staged in LDS at a time (64 per wave)
constexpr int kMaxL = 64;                     // largest L array (LDS: kMaxL * 256 * 8 B)
constexpr int kMaxAnt = 512;                  // T + R
constexpr int kSortChunk = 16384;             // rows sorted by one work-group
constexpr int kSortThreads = 1024;
constexpr int kMaxB = 1 << 24;

struct Geo {
    const double *ant;    // (T + R) x 3 positions, transmitters first
    const double *kappa;  // F: f / c in turns per metre
    const float2 *q;      // F: p(f) / (4 pi)
    int T, R, F;
    int nx, ny, nz;
    int nbx, nby, nbz;    // bricks per axis
    int g_is_tx;          // 1: G = transmitters, L = receivers
    int nG, nL;
    double cx, cy, cz;    // grid centre
    double px, py, pz;    // pitch
    // Precomputed L-side tables of the plan's phase policy, [brick][nL][256] entries of 8 bytes
    // (nullptr: every work-group forms its brick's table itself); ltab_mode names the policy.
    const float4 *ltab;
    int ltab_mode;
};

// ------------------------------------------------------------------------------------------
// Device helpers
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum sixteen per-lane values x[q] (one per row q) over the 64 lanes of a wave at once.  Each
// halving step swaps half of the lanes between two registers and adds, so that the number of
// live registers halves while the lanes summed into each doubles (32-lane and 16-lane swaps,
// then an 8-lane rotation and a 4-lane mirror inside each 16-lane row, then a quad sum).  On
// return lane l holds the total of row l >> 2.  b3, b2: bits 3 and 2 of the lane index.
__device__ __forceinline__ float wave_transpose_sum16(const float (&x)[16], bool b3, bool b2) {
    float y[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[j]), __float_as_uint(x[j + 8]), false, false);
        y[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);  // lanes 0-31: row j, 32-63: row j+8
    }
    float z[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(y[j]), __float_as_uint(y[j + 4]), false, false);
        z[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);  // 16-lane group g: row j + 4g
    }
    float w[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const float t1 = b3 ? z[j + 2] : z[j];
        const float t2 = b3 ? z[j] : z[j + 2];
        w[j] = t1 + dpp_f<0x128>(t2);  // row_ror:8; bit3 = 0: row j + 4g, bit3 = 1: row j + 2 + 4g
    }
    const float t1 = b2 ? w[1] : w[0];
    const float t2 = b2 ? w[0] : w[1];
    float v = t1 + dpp_f<0x141>(t2);   // row_half_mirror; row 4g + 2 bit3 + bit2 = l >> 2
    v += dpp_f<0xB1>(v);                // quad_perm [1,0,3,2]
    v += dpp_f<0x4E>(v);                // quad_perm [2,3,0,1]
    return v;
}

// Brick decomposition of a tile index.
__device__ __forceinline__ void brick_of(const Geo &g, int tile, int &bx, int &by, int &bz) {
    bx = tile % g.nbx;
    by = (tile / g.nbx) % g.nby;
    bz = tile / (g.nbx * g.nby);
}

// Offset of local voxel (lx, ly, lz) from the brick centre, metres, float32.
__device__ __forceinline__ void local_offset(const Geo &g, int lx, int ly, int lz, float &ex, float &ey,
                                             float &ez) {
    ex = (float)((lx - 0.5 * (kBX - 1)) * g.px);
    ey = (float)((ly - 0.5 * (kBY - 1)) * g.py);
    ez = (float)((lz - 0.5 * (kBZ - 1)) * g.pz);
}

// Distance offset delta = d_{a,n} - d_{a,c} and amplitude w = 1/d_{a,n} for a voxel at offset e
// from the brick centre; ga = (c - r_a, |c - r_a|) in float32.
__device__ __forceinline__ void comp_offset(float ex, float ey, float ez, float4 ga, float &delta, float &w) {
    const float vx = ex + ga.x, vy = ey + ga.y, vz = ez + ga.z;
    const float d2 = fmaf(vx, vx, fmaf(vy, vy, vz * vz));
    const float d = sqrtf(d2);
    const float ee = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
    const float num = fmaf(2.0f, fmaf(ex, ga.x, fmaf(ey, ga.y, ez * ga.z)), ee);
    delta = num / (d + ga.w);
    w = 1.0f / d;
}

// Same quantities with hardware reciprocal square root / reciprocal, each refined by one Newton
// step (relative error about 1e-7, like the correctly rounded forms, at a third of the cost).
__device__ __forceinline__ void comp_offset_fast(float ex, float ey, float ez, float ee, float4 ga, float &delta,
                                                 float &w) {
    const float vx = ex + ga.x, vy = ey + ga.y, vz = ez + ga.z;
    const float d2 = fmaf(vx, vx, fmaf(vy, vy, vz * vz));
    float r = __builtin_amdgcn_rsqf(d2);
    r = r * fmaf(-0.5f * d2 * r, r, 1.5f);            // Newton step for 1/sqrt(d2)
    const float d = d2 * r;
    const float den = d + ga.w;
    float inv = __builtin_amdgcn_rcpf(den);
    inv = inv * fmaf(-den, inv, 2.0f);                // Newton step for 1/den
    const float num = fmaf(2.0f, fmaf(ex, ga.x, fmaf(ey, ga.y, ez * ga.z)), ee);
    delta = num * inv;
    w = r;
}

// Decode measurement index m = (f*T + t)*R + r into (f, G index, L index).
__device__ __forceinline__ void decode_row(const Geo &g, int m, int &f, int &gi, int &li) {
    const int r = m % g.R;
    const int t = (m / g.R) % g.T;
    f = m / (g.R * g.T);
    gi = g.g_is_tx ? t : r;
    li = g.g_is_tx ? r : t;
}

__device__ __forceinline__ int ant_of_g(const Geo &g, int gi) { return g.g_is_tx ? gi : g.T + gi; }
__device__ __forceinline__ int ant_of_l(const Geo &g, int li) { return g.g_is_tx ? g.T + li : li; }

// ------------------------------------------------------------------------------------------
// 1. Sort the minibatch by (G, L, f, original position), one work-group per chunk of rows.
//    Output srt[i] = (original position j, f, G index, L index) of the i-th sorted row.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void sort_rows_body(const Geo &g, unsigned long long *keys, const int32_t *__restrict__ rows,
                                               int B, int4 *__restrict__ srt, int *__restrict__ status, int chunk) {
    const int c0 = chunk * kSortChunk;
    const int n = min(kSortChunk, B - c0);
    int p2 = 2;
    while (p2 < n) p2 <<= 1;
    const int M = g.F * g.T * g.R;
    for (int i = threadIdx.x; i < p2; i += kSortThreads) {
        unsigned long long key = ~0ull;
        if (i < n) {
            int m = rows[c0 + i];
            if (m < 0 || m >= M) {
                atomicOr(status, 1);
                m = 0;
            }
            int f, gi, li;
            decode_row(g, m, f, gi, li);
            const unsigned int pk = (unsigned int)((gi * g.nL + li) * g.F + f);
            key = ((unsigned long long)pk << 32) | (unsigned int)i;
        }
        keys[i] = key;
    }
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < p2; i += kSortThreads) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const unsigned long long a = keys[i], b = keys[ixj];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        keys[i] = b;
                        keys[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < n; i += kSortThreads) {
        const unsigned long long key = keys[i];
        const int j = (int)(key & 0xffffffffu);
        const unsigned int pk = (unsigned int)(key >> 32);
        const int f = (int)(pk % (unsigned int)g.F);
        const unsigned int pair = pk / (unsigned int)g.F;
        const int li = (int)(pair % (unsigned int)g.nL);
        const int gi = (int)(pair / (unsigned int)g.nL);
        srt[c0 + i] = make_int4(c0 + j, f, gi, li);
    }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_rows(Geo g, const int32_t *__restrict__ rows, int B,
                                                            int4 *__restrict__ srt, int *__restrict__ status) {
    extern __shared__ unsigned long long keys[];  // next power of two >= min(B, kSortChunk)
    // minibatch blockIdx.y of a batched sort
    sort_rows_body(g, keys, rows + (size_t)blockIdx.y * B, B, srt + (size_t)blockIdx.y * B, status, blockIdx.x);
}

// ------------------------------------------------------------------------------------------
// Shared prologue of the two tile kernels: antenna terms relative to the brick centre and the
// L-side per-voxel terms, staged in LDS.
// ------------------------------------------------------------------------------------------
struct TileSmem {
    float4 *antg;    // [T+R]: COMP32 (c - r_a, |c - r_a|) / NAIVE32 (r_a, 0), float32
    double *antd;    // [T+R]: COMP32 |c - r_a| float64
    double4 *antg64; // [T+R]: F64 (c - r_a, |c - r_a|) float64 (aliases antg/antd)
    float4 *rowinfo; // [kSub]: (row data x, row data y, packed row word as bits, 0)
    float2 *rowv;    // [kSub]: forward row sums / adjoint scaled residuals
    float2 *snew;    // [kBrick]: the brick's iterate after a deferred proximal step (forward)
    void *lside;     // [nL][256]: per L antenna per brick voxel (layout set by the phase policy)
};

// Packed row word: G index (bits 0-11), L index (bits 12-23), and two flags telling whether the
// row starts a new G antenna or a new (G, L) pair relative to the previous row of the same wave.
constexpr int kNewG = 1 << 30;
constexpr int kNewPair = 1 << 29;
__device__ __forceinline__ int row_g(int w) { return w & 0xfff; }
__device__ __forceinline__ int row_l(int w) { return (w >> 12) & 0xfff; }

constexpr size_t kAntBytes = 32;  // LDS bytes per antenna (largest policy)

// LDS carve-up of a tile work-group of W waves (W x 64 rows staged per sub-chunk).
template <int W = kWaves>
__device__ __forceinline__ TileSmem carve(char *smem, const Geo &g) {
    constexpr int sub = W * kWave;
    TileSmem t;
    const int A = g.T + g.R;
    t.antg = reinterpret_cast<float4 *>(smem);
    t.antd = reinterpret_cast<double *>(smem + sizeof(float4) * A);
    t.antg64 = reinterpret_cast<double4 *>(smem);
    char *p = smem + kAntBytes * A;
    t.rowinfo = reinterpret_cast<float4 *>(p);
    t.rowv = reinterpret_cast<float2 *>(t.rowinfo + sub);
    t.snew = t.rowv + sub;
    t.lside = t.snew + kBrick;
    return t;
}

__device__ __forceinline__ void brick_centre(const Geo &g, int bx, int by, int bz, double &cx, double &cy,
                                             double &cz) {
    cx = g.cx + (bx * kBX + 0.5 * (kBX - 1) - 0.5 * (g.nx - 1)) * g.px;
    cy = g.cy + (by * kBY + 0.5 * (kBY - 1) - 0.5 * (g.ny - 1)) * g.py;
    cz = g.cz + (bz * kBZ + 0.5 * (kBZ - 1) - 0.5 * (g.nz - 1)) * g.pz;
}

// ------------------------------------------------------------------------------------------
// Phase policies.  Each turns the geometry of a (row, voxel) pair into the float32 phase in
// turns that feeds v_sin_f32 / v_cos_f32, and supplies the amplitude 1/(d_G d_L).
//   G state: per lane voxel, rebuilt when the G antenna changes (registers);
//   L entry: per (L antenna, brick voxel), staged once per brick (LDS);
//   D      : per lane voxel, the pair's distance term (G state + L entry);
//   row data (x, y): per row, from f/c and the brick's reference distances.
// ------------------------------------------------------------------------------------------
template <int MODE> struct Phase;

// Compensated float32 (default): offsets from the brick centre, float64 per-row reference.
template <> struct Phase<SPGM_PHASE_COMP32> {
    using D = float;
    using LE = float2;  // (delta, 1/d)
    struct Vox { float ex, ey, ez, ee; };
    static __device__ Vox vox(const Geo &g, int bx, int by, int bz, int lx, int ly, int lz) {
        Vox v;
        local_offset(g, lx, ly, lz, v.ex, v.ey, v.ez);
        v.ee = fmaf(v.ex, v.ex, fmaf(v.ey, v.ey, v.ez * v.ez));
        return v;
    }
    static __device__ void stage_ant(const Geo &g, const TileSmem &sm, int a, double cx, double cy, double cz) {
        const double gx = cx - g.ant[3 * a], gy = cy - g.ant[3 * a + 1], gz = cz - g.ant[3 * a + 2];
        const double d = sqrt(gx * gx + gy * gy + gz * gz);
        sm.antd[a] = d;
        sm.antg[a] = make_float4((float)gx, (float)gy, (float)gz, (float)d);
    }
    static __device__ void geom(const TileSmem &sm, int a, const Vox &v, D &d, float &w) {
        comp_offset_fast(v.ex, v.ey, v.ez, v.ee, sm.antg[a], d, w);
    }
    static __device__ LE lentry(D d, float w) { return make_float2(d, w); }
    static __device__ D pair_d(D dg, LE le) { return dg + le.x; }
    static __device__ float lw(LE le) { return le.y; }
    static __device__ float2 row_data(const TileSmem &sm, double kap, int ga, int la) {
        double ph = kap * (sm.antd[ga] + sm.antd[la]);
        ph -= rint(ph);
        return make_float2((float)kap, (float)ph);
    }
    static __device__ float phase(float4 ri, D d) { return fmaf(ri.x, d, ri.y); }
};

// Float64 distances and phase, reduced modulo one turn in float64, then float32 sin/cos.
template <> struct Phase<SPGM_PHASE_F64> {
    using D = double;
    using LE = double;  // d
    struct Vox { double ex, ey, ez; };
    static __device__ Vox vox(const Geo &g, int bx, int by, int bz, int lx, int ly, int lz) {
        Vox v;
        v.ex = (lx - 0.5 * (kBX - 1)) * g.px;
        v.ey = (ly - 0.5 * (kBY - 1)) * g.py;
        v.ez = (lz - 0.5 * (kBZ - 1)) * g.pz;
        return v;
    }
    static __device__ void stage_ant(const Geo &g, const TileSmem &sm, int a, double cx, double cy, double cz) {
        const double gx = cx - g.ant[3 * a], gy = cy - g.ant[3 * a + 1], gz = cz - g.ant[3 * a + 2];
        sm.antg64[a] = make_double4(gx, gy, gz, 0.0);
    }
    static __device__ void geom(const TileSmem &sm, int a, const Vox &v, D &d, float &w) {
        const double4 ga = sm.antg64[a];
        const double x = v.ex + ga.x, y = v.ey + ga.y, z = v.ez + ga.z;
        d = sqrt(fma(x, x, fma(y, y, z * z)));
        w = (float)(1.0 / d);
    }
    static __device__ LE lentry(D d, float) { return d; }
    static __device__ D pair_d(D dg, LE le) { return dg + le; }
    static __device__ float lw(LE le) { return __builtin_amdgcn_rcpf((float)le); }
    static __device__ float2 row_data(const TileSmem &, double kap, int, int) {
        return make_float2(__int_as_float(__double2loint(kap)), __int_as_float(__double2hiint(kap)));
    }
    static __device__ float phase(float4 ri, D d) {
        const double kap = __hiloint2double(__float_as_int(ri.y), __float_as_int(ri.x));
        const double ph = kap * d;
        return (float)(ph - floor(ph));
    }
};

// Uncompensated float32: absolute float32 positions, float32 distance and phase.
template <> struct Phase<SPGM_PHASE_NAIVE32> {
    using D = float;
    using LE = float2;  // (d, 1/d)
    struct Vox { float x, y, z; };
    static __device__ Vox vox(const Geo &g, int bx, int by, int bz, int lx, int ly, int lz) {
        Vox v;
        v.x = (float)(g.cx + (bx * kBX + lx - 0.5 * (g.nx - 1)) * g.px);
        v.y = (float)(g.cy + (by * kBY + ly - 0.5 * (g.ny - 1)) * g.py);
        v.z = (float)(g.cz + (bz * kBZ + lz - 0.5 * (g.nz - 1)) * g.pz);
        return v;
    }
    static __device__ void stage_ant(const Geo &g, const TileSmem &sm, int a, double, double, double) {
        sm.antg[a] = make_float4((float)g.ant[3 * a], (float)g.ant[3 * a + 1], (float)g.ant[3 * a + 2], 0.f);
    }
    static __device__ void geom(const TileSmem &sm, int a, const Vox &v, D &d, float &w) {
        const float4 ra = sm.antg[a];
        const float x = v.x - ra.x, y = v.y - ra.y, z = v.z - ra.z;
        d = sqrtf(fmaf(x, x, fmaf(y, y, z * z)));
        w = 1.0f / d;
    }
    static __device__ LE lentry(D d, float w) { return make_float2(d, w); }
    static __device__ D pair_d(D dg, LE le) { return dg + le.x; }
    static __device__ float lw(LE le) { return le.y; }
    static __device__ float2 row_data(const TileSmem &, double kap, int, int) {
        return make_float2((float)kap, 0.f);
    }
    static __device__ float phase(float4 ri, D d) { return __builtin_amdgcn_fractf(ri.x * d); }
};

// Antenna terms of brick (bx, by, bz) and its L-side table in LDS.  With a precomputed table
// for this policy the brick's entries are copied (16-byte loads) instead of formed; either way
// the caller synchronises the work-group before reading them.
template <int MODE, bool TABLE = true>
__device__ __forceinline__ void stage_tile(const Geo &g, const TileSmem &sm, int bx, int by, int bz) {
    using P = Phase<MODE>;
    static_assert(sizeof(typename P::LE) == 8, "L-side entries are 8 bytes");
    double cx, cy, cz;
    brick_centre(g, bx, by, bz, cx, cy, cz);
    const int A = g.T + g.R;
    const int nthr = blockDim.x;  // a multiple of kBrick
    for (int a = threadIdx.x; a < A; a += nthr) P::stage_ant(g, sm, a, cx, cy, cz);
    if (TABLE && g.ltab && g.ltab_mode == MODE) {
        const int n4 = g.nL * (kBrick / 2);  // float4 per brick table
        const float4 *src = g.ltab + (size_t)((bz * g.nby + by) * g.nbx + bx) * n4;
        float4 *dst = static_cast<float4 *>(sm.lside);
        for (int i = threadIdx.x; i < n4; i += nthr) dst[i] = src[i];
        return;
    }
    __syncthreads();
    const int v = threadIdx.x % kBrick;  // brick voxel: lane -> (x, y), (wave mod 4) -> z
    const int lx = (v & 63) & 7, ly = (v & 63) >> 3, lz = v >> 6;
    const bool inside = bx * kBX + lx < g.nx && by * kBY + ly < g.ny && bz * kBZ + lz < g.nz;
    const typename P::Vox vx = P::vox(g, bx, by, bz, lx, ly, lz);
    typename P::LE *lside = static_cast<typename P::LE *>(sm.lside);
    for (int li = threadIdx.x / kBrick; li < g.nL; li += nthr / kBrick) {
        typename P::D dl = 0;
        float wl = 0.f;
        if (inside) P::geom(sm, ant_of_l(g, li), vx, dl, wl);
        lside[li * kBrick + v] = P::lentry(dl, wl);  // voxels outside the grid contribute 0
    }
}

// Forms the L-side table of brick blockIdx.x with the same code as stage_tile and stores it.
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_build_ltab(Geo g, float4 *__restrict__ tab) {
    extern __shared__ __align__(16) char smem[];
    const TileSmem sm = carve(smem, g);
    int bx, by, bz;
    brick_of(g, blockIdx.x, bx, by, bz);
    stage_tile<MODE, false>(g, sm, bx, by, bz);
    __syncthreads();
    const int n4 = g.nL * (kBrick / 2);
    const float4 *src = static_cast<const float4 *>(sm.lside);
    float4 *dst = tab + (size_t)blockIdx.x * n4;
    for (int i = threadIdx.x; i < n4; i += kThreads) dst[i] = src[i];
}

// Order a wave's own LDS accesses across this point.  A wave's LDS instructions execute in
// issue order, so data written by one lane is seen by later reads of any lane of the same wave;
// only the compiler has to be kept from moving accesses across (no work-group barrier needed).
__device__ __forceinline__ void wave_lds_order() { asm volatile("" ::: "memory"); }

// Brick and row split of a tile work-group on a (bricks, splits) grid.  Work-groups go to the
// eight XCDs round-robin in linear launch order; when the brick count is a multiple of eight,
// consecutive work-groups on one XCD take the row splits of one brick, so the splits read that
// brick's L-side table and source values through the same L2 at about the same time instead of
// once per split from the fabric.  Otherwise the grid coordinates are used directly.
__device__ __forceinline__ void tile_and_split(int &tile, int &split) {
    const int nt = gridDim.x, ns = gridDim.y;
    if ((nt & 7) != 0) {
        tile = blockIdx.x;
        split = blockIdx.y;
        return;
    }
    const int lin = blockIdx.y * nt + blockIdx.x;
    const int slot = lin >> 3, q = slot / ns;
    tile = (lin & 7) + 8 * q;
    split = slot - q * ns;
}

// Each wave owns a contiguous run of the work-group's sorted rows [r0, r1): wave w takes
// [wb, we), a multiple of 64 rows long, so antenna changes stay as rare as in the sorted order.
template <int W = kWaves>
__device__ __forceinline__ void wave_rows(int r0, int r1, int w, int &wb, int &we, int &nsub) {
    const int per = ((r1 - r0 + W - 1) / W + kWave - 1) / kWave * kWave;
    wb = min(r1, r0 + w * per);
    we = min(r1, wb + per);
    nsub = per / kWave;  // sub-chunks of 64 rows per wave (same for every wave)
}

// Global part of staging sub-chunk j: thread t holds row wb(t/64) + 64 j + t%64 of its wave's
// run; it loads that sorted row and its predecessor's antennas (pg = -1 for the first row of the
// run, r = -1 past its end).  Issued one sub-chunk ahead, the loads are in flight while the rows
// of the current sub-chunk are processed.
struct RowFetch {
    int r, pg, pl;
    int4 info;
};

template <int W = kWaves>
__device__ __forceinline__ RowFetch fetch_rows(const int4 *__restrict__ srt, int r0, int r1, int j) {
    const int t = threadIdx.x;
    int wb, we, nsub;
    wave_rows<W>(r0, r1, t / kWave, wb, we, nsub);
    RowFetch f;
    f.r = wb + j * kWave + (t % kWave);
    f.pg = f.pl = -1;
    f.info = make_int4(0, 0, 0, 0);
    if (f.r >= we) {
        f.r = -1;
        return f;
    }
    f.info = srt[f.r];
    if (f.r > wb) {
        const int4 prev = srt[f.r - 1];
        f.pg = prev.z;
        f.pl = prev.w;
    }
    return f;
}

// Stage a fetched sub-chunk into LDS.  Returns the sorted row index (or -1).  Row data: the
// policy's two words (f/c and the per-brick reference phase for COMP32) and the packed row word.
template <int MODE>
__device__ __forceinline__ int stage_fetched(const Geo &g, const TileSmem &sm, const RowFetch &f) {
    if (f.r < 0) return -1;
    const int4 info = f.info;
    const float2 rd = Phase<MODE>::row_data(sm, g.kappa[info.y], ant_of_g(g, info.z), ant_of_l(g, info.w));
    int word = info.z | (info.w << 12);
    if (f.pg != info.z) word |= kNewG | kNewPair;  // also the first row of the run (pg = -1)
    else if (f.pl != info.w) word |= kNewPair;
    sm.rowinfo[threadIdx.x] = make_float4(rd.x, rd.y, __int_as_float(word), 0.f);
    return f.r;
}

// Fixed-order sum over the row splits of the adjoint partials of voxel n (four loads in
// flight, then the additions in order).
__device__ __forceinline__ float2 split_sum(const float2 *__restrict__ gpart, int nsplit, int N, size_t n) {
    float gr = 0.f, gi = 0.f;
    int k = 0;
    for (; k + 3 < nsplit; k += 4) {
        float2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = gpart[(size_t)(k + u) * N + n];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            gr += v[u].x;
            gi += v[u].y;
        }
    }
    for (; k < nsplit; ++k) {
        const float2 v = gpart[(size_t)k * N + n];
        gr += v.x;
        gi += v.y;
    }
    return make_float2(gr, gi);
}

// Gradient step and complex soft threshold of Eq. 5: S_alpha(v - step g).
__device__ __forceinline__ float2 prox_step(float2 v, float2 g, float step, float alpha) {
    v.x = fmaf(-step, g.x, v.x);
    v.y = fmaf(-step, g.y, v.y);
    const float mag = sqrtf(fmaf(v.x, v.x, v.y * v.y));
    if (mag <= alpha) return make_float2(0.f, 0.f);
    const float sc = 1.0f - alpha / mag;
    return make_float2(v.x * sc, v.y * sc);
}

// The previous iteration's proximal step, deferred into the forward: the forward applies it to
// the voxels it reads, s_k = S_alpha(s_{k-1} - step sum_splits gpart) (the column reduction's
// arithmetic), and the work-groups of row split 0 store s_k to s_out, which must not alias the
// s_{k-1} the other splits read.  gpart == nullptr: s is used as given.
struct SStep {
    const float2 *gpart;
    float2 *s_out;
    int nsplit, N;
    float step, alpha;
};

// ------------------------------------------------------------------------------------------
// 2. Forward partials: part[tile][i] = sum over brick voxels of (A_{row i, n} / q_f) s_n.
// ------------------------------------------------------------------------------------------
// Body shared by the single-plan launch (one brick x row range per work-group) and the
// work-list launch over many scenes: brick `tile`, sorted rows [r0, r1).
template <int MODE, int W = kWaves>
__device__ __forceinline__ void fwd_tile_body(const Geo &g, char *smem, int tile, int r0, int r1,
                                              const int4 *__restrict__ srt, int B, const float2 *s,
                                              float2 *__restrict__ part, const SStep &up, bool store_s) {
    using P = Phase<MODE>;
    using DT = typename P::D;
    const TileSmem sm = carve<W>(smem, g);
    int bx, by, bz;
    brick_of(g, tile, bx, by, bz);
    // A deferred proximal step: the first four waves form the brick's new iterate (voxel
    // p * 64 + lane) into LDS, where the lanes read it after the barrier below.
    const bool deferred = up.gpart != nullptr;
    if (deferred && threadIdx.x < kBrick) {
        const int v = threadIdx.x, ln = v & 63;
        const int jx = bx * kBX + (ln & 7), jy = by * kBY + (ln >> 3), jz = bz * kBZ + (v >> 6);
        float2 val = make_float2(0.f, 0.f);
        if (jx < g.nx && jy < g.ny && jz < g.nz) {
            const size_t n = ((size_t)jz * g.ny + jy) * g.nx + jx;
            val = prox_step(s[n], split_sum(up.gpart, up.nsplit, up.N, n), up.step, up.alpha);
            if (store_s) up.s_out[n] = val;
        }
        sm.snew[v] = val;
    }
    stage_tile<MODE>(g, sm, bx, by, bz);

    const int lane = threadIdx.x & 63;
    const int wave = uniform(threadIdx.x >> 6);  // wave-uniform: keeps row loops on the scalar unit
    const int lx = lane & 7, ly = lane >> 3;
    const int ix = bx * kBX + lx, iy = by * kBY + ly;
    typename P::Vox vox[kP];
    float sr[kP], si[kP];
    bool valid[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        const int iz = bz * kBZ + p;
        valid[p] = ix < g.nx && iy < g.ny && iz < g.nz;
        vox[p] = P::vox(g, bx, by, bz, lx, ly, p);
        float2 sv = make_float2(0.f, 0.f);
        if (!deferred && valid[p]) sv = s[((size_t)iz * g.ny + iy) * g.nx + ix];
        sr[p] = sv.x;
        si[p] = sv.y;
    }
    const typename P::LE *lbase = static_cast<const typename P::LE *>(sm.lside) + lane;  // + li * kBrick + p * kWave

    DT dG[kP], D[kP];
    float usr[kP], usi[kP], ur[kP], ui[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        dG[p] = D[p] = 0;
        usr[p] = usi[p] = ur[p] = ui[p] = 0.f;
    }
    float accr[16], acci[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) accr[q] = acci[q] = 0.f;
    const bool b3 = lane & 8, b2 = lane & 4;
    int wb, we, nsub;
    wave_rows<W>(r0, r1, wave, wb, we, nsub);
    const float4 *rinfo = sm.rowinfo + wave * kWave;

    // Every wave stages, reads and stores only its own rows, so after the brick tables are
    // staged the waves run their row loops independently (no work-group barrier per sub-chunk).
    RowFetch next = fetch_rows<W>(srt, r0, r1, 0);
    __syncthreads();  // brick tables (and a deferred step's iterate) staged
    if (deferred) {
#pragma unroll
        for (int p = 0; p < kP; ++p) {
            const float2 sv = sm.snew[p * kWave + lane];
            sr[p] = sv.x;
            si[p] = sv.y;
        }
    }
    for (int j = 0; j < nsub; ++j) {
        wave_lds_order();  // previous sub-chunk's row data consumed
        const int my_row = stage_fetched<MODE>(g, sm, next);
        wave_lds_order();
        if (j + 1 < nsub) next = fetch_rows<W>(srt, r0, r1, j + 1);
        const int cnt = max(0, min(kWave, we - wb - j * kWave));
        // Blocks of 16 consecutive rows, one transposed reduction each.  G-antenna and pair changes
        // are handled at the row where they happen.  Rows of the last block past cnt are formed
        // from stale entries of this wave's row buffer (i0 + 15 < 64) and discarded: the
        // transposed reduction never mixes rows, and their flags are masked off, so they change
        // no state.
        for (int i0 = 0; i0 < cnt; i0 += 16) {
            const int len = min(16, cnt - i0);
            const int q = lane & 15;
            const int wq = __float_as_int(rinfo[i0 + min(q, len - 1)].z);  // lane q: word of row i0 + q
            // pair changes of the block as a scalar bit mask: the per-row branch needs no lane read
            const unsigned long long live = len == 16 ? 0xffffull : (1ull << len) - 1;
            const unsigned long long pairs = __ballot(wq & kNewPair) & live;
            // The block's row entries are read through one address register with immediate
            // offsets: an opaque zero keeps the base in a VGPR instead of re-forming it per row.
            int zero;
            asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
            const float4 *rblk = rinfo + i0 + zero;
#pragma unroll
            for (int qq = 0; qq < 16; ++qq) {
                const float4 ri = rblk[qq];
                if ((pairs >> qq) & 1ull) {
                    const int word = __builtin_amdgcn_readlane(wq, qq);
                    if (word & kNewG) {  // a new G antenna also starts a new pair
                        const int ga = ant_of_g(g, row_g(word));
#pragma unroll
                        for (int p = 0; p < kP; ++p) {
                            DT dg;
                            float wg;
                            P::geom(sm, ga, vox[p], dg, wg);
                            dG[p] = valid[p] ? dg : DT(0);
                            usr[p] = valid[p] ? wg * sr[p] : 0.f;
                            usi[p] = valid[p] ? wg * si[p] : 0.f;
                        }
                    }
                    const typename P::LE *lp = lbase + row_l(word) * kBrick;
#pragma unroll
                    for (int p = 0; p < kP; ++p) {
                        const typename P::LE lv = lp[p * kWave];
                        const float wl = P::lw(lv);
                        D[p] = P::pair_d(dG[p], lv);
                        ur[p] = wl * usr[p];
                        ui[p] = wl * usi[p];
                    }
                }
                float ar, ai;
#pragma unroll
                for (int p = 0; p < kP; ++p) {
                    const float ph = P::phase(ri, D[p]);
                    const float sn = __builtin_amdgcn_sinf(ph);
                    const float cs = __builtin_amdgcn_cosf(ph);
                    // (cs - j sn)(ur + j ui)
                    if (p == 0) {
                        ar = cs * ur[p];
                        ai = cs * ui[p];
                    } else {
                        ar = fmaf(cs, ur[p], ar);
                        ai = fmaf(cs, ui[p], ai);
                    }
                    ar = fmaf(sn, ui[p], ar);
                    ai = fmaf(-sn, ur[p], ai);
                }
                // the row's sums are formed here, not sunk to the reduction (which would keep every
                // row's pair terms live at once)
                asm volatile("" : "+v"(ar), "+v"(ai));
                accr[qq] = ar;
                acci[qq] = ai;
            }
            const float tr = wave_transpose_sum16(accr, b3, b2);
            const float ti = wave_transpose_sum16(acci, b3, b2);
            const int row = lane >> 2;
            if ((lane & 3) == 0 && row < len) sm.rowv[wave * kWave + i0 + row] = make_float2(tr, ti);
        }
        wave_lds_order();
        if (my_row >= 0) part[(size_t)tile * B + my_row] = sm.rowv[threadIdx.x];
    }
}

template <int MODE, int W>
__global__ __launch_bounds__(W * 64) void k_fwd_tile(Geo g, const int4 *__restrict__ srt, int B, int rows_per_wg,
                                                     const float2 *s, float2 *__restrict__ part, SStep up) {
    extern __shared__ __align__(16) char smem[];
    int tile, split;
    tile_and_split(tile, split);
    const int r0 = split * rows_per_wg;
    fwd_tile_body<MODE, W>(g, smem, tile, r0, min(B, r0 + rows_per_wg), srt, B, s, part, up, split == 0);
}

// ------------------------------------------------------------------------------------------
// 3. Row reduction: v_i = q_f * sum_tiles part[tile][i]  (minus y_m when y is given).
//    out_user[j] = v (caller order); out_scaled[i] = conj(q_f) * v (sorted order, adjoint input).
// ------------------------------------------------------------------------------------------
constexpr int kRedGroups = 16;  // tile groups per row-reduction work-group (ROWS rows x 16)
constexpr int kRedRows = 16;    // rows per work-group of the single-plan reduction

// ROWS rows per work-group of ROWS * kRedGroups threads; thread group k sums the tiles
// t = k mod kRedGroups and the groups are combined in order, whatever ROWS is.
template <int ROWS>
__device__ __forceinline__ void row_reduce_body(const Geo &g, const float2 *__restrict__ part, int n_tiles, int B,
                                                const int4 *__restrict__ srt, const int32_t *__restrict__ rows,
                                                const float2 *__restrict__ y, float2 *__restrict__ out_user,
                                                float2 *__restrict__ out_scaled, int row0) {
    __shared__ float2 red[kRedGroups][ROWS];
    const int tx = threadIdx.x % ROWS, ty = threadIdx.x / ROWS;
    const int i = row0 + tx;
    float ar = 0.f, ai = 0.f;
    if (i < B) {
        // eight loads in flight, then the additions in tile order
        int t = ty;
        for (; t + 7 * kRedGroups < n_tiles; t += 8 * kRedGroups) {
            float2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(t + u * kRedGroups) * B + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                ar += v[u].x;
                ai += v[u].y;
            }
        }
        for (; t < n_tiles; t += kRedGroups) {
            const float2 v = part[(size_t)t * B + i];
            ar += v.x;
            ai += v.y;
        }
    }
    red[ty][tx] = make_float2(ar, ai);
    __syncthreads();
    if (ty == 0 && i < B) {
        ar = red[0][tx].x;
        ai = red[0][tx].y;
        for (int k = 1; k < kRedGroups; ++k) {
            ar += red[k][tx].x;
            ai += red[k][tx].y;
        }
        const int4 info = srt[i];
        const float2 q = g.q[info.y];
        float vr = q.x * ar - q.y * ai;
        float vi = q.x * ai + q.y * ar;
        if (y) {
            int m = rows[info.x];
            const int M = g.F * g.T * g.R;
            if (m < 0 || m >= M) m = 0;
            const float2 ym = y[m];
            vr -= ym.x;
            vi -= ym.y;
        }
        if (out_user) out_user[info.x] = make_float2(vr, vi);
        if (out_scaled) out_scaled[i] = make_float2(q.x * vr + q.y * vi, q.x * vi - q.y * vr);
    }
}

// Few rows per work-group, so that even a few thousand rows spread over every compute unit.
__global__ __launch_bounds__(kRedRows * kRedGroups) void k_row_reduce(Geo g, const float2 *__restrict__ part,
                                                                     int n_tiles, int B,
                                                                     const int4 *__restrict__ srt,
                                                                     const int32_t *__restrict__ rows,
                                                                     const float2 *__restrict__ y,
                                                                     float2 *__restrict__ out_user,
                                                                     float2 *__restrict__ out_scaled) {
    row_reduce_body<kRedRows>(g, part, n_tiles, B, srt, rows, y, out_user, out_scaled, blockIdx.x * kRedRows);
}

// Adjoint input for a caller-supplied residual: out_scaled[i] = conj(q_f) * r[j_i].
__global__ __launch_bounds__(256) void k_gather_scale(Geo g, const int4 *__restrict__ srt, int B,
                                                      const float2 *__restrict__ r, float2 *__restrict__ out_scaled) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B) {
        const int4 info = srt[i];
        const float2 q = g.q[info.y];
        const float2 v = r[info.x];
        out_scaled[i] = make_float2(q.x * v.x + q.y * v.y, q.x * v.y - q.y * v.x);
    }
}

// ------------------------------------------------------------------------------------------
// 4. Adjoint partials: gpart[split][n] = sum over the split's rows of conj(A_{i,n}/q_f) rs_i,
//    with rs_i = conj(q_f) r_i, one voxel column per lane, rows shared by the eight waves.
//    Rows of one (G, L) pair share the amplitude 1/(d_G d_L) of each voxel, so their terms are
//    summed first and scaled once when the pair ends.
// ------------------------------------------------------------------------------------------
template <int MODE, int W = kWaves>
__device__ __forceinline__ void adj_tile_body(const Geo &g, char *smem, int tile, int split, int r0, int r1,
                                              const int4 *__restrict__ srt, int B, const float2 *__restrict__ rs,
                                              float2 *__restrict__ gpart, int N) {
    using P = Phase<MODE>;
    using DT = typename P::D;
    const TileSmem sm = carve<W>(smem, g);
    int bx, by, bz;
    brick_of(g, tile, bx, by, bz);
    stage_tile<MODE>(g, sm, bx, by, bz);

    const int lane = threadIdx.x & 63;
    const int wave = uniform(threadIdx.x >> 6);  // wave-uniform: keeps row loops on the scalar unit
    const int lx = lane & 7, ly = lane >> 3;
    typename P::Vox vox[kP];
    bool valid[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        vox[p] = P::vox(g, bx, by, bz, lx, ly, p);
        valid[p] = bx * kBX + lx < g.nx && by * kBY + ly < g.ny && bz * kBZ + p < g.nz;
    }
    const typename P::LE *lbase = static_cast<const typename P::LE *>(sm.lside) + lane;

    DT dG[kP], D[kP];
    float wG[kP], Wpr[kP], hr[kP], hi[kP], gr[kP], gi_[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        dG[p] = D[p] = 0;
        wG[p] = Wpr[p] = hr[p] = hi[p] = gr[p] = gi_[p] = 0.f;
    }
    int wb, we, nsub;
    wave_rows<W>(r0, r1, wave, wb, we, nsub);
    const float4 *rinfo = sm.rowinfo + wave * kWave;

    RowFetch next = fetch_rows<W>(srt, r0, r1, 0);
    __syncthreads();  // brick tables staged; from here each wave works on its own rows only
    for (int j = 0; j < nsub; ++j) {
        wave_lds_order();  // previous sub-chunk's row data consumed
        const int my_row = stage_fetched<MODE>(g, sm, next);
        // Row data for the loop: (policy words, residual) in one LDS entry per row; the row word
        // stays in this lane's register and the pair changes of the sub-chunk become a scalar bit
        // mask, so the per-row branch waits for no LDS read.
        int my_word = 0;
        if (my_row >= 0) {
            float4 e = sm.rowinfo[threadIdx.x];
            my_word = __float_as_int(e.z);
            const float2 rv = rs[my_row];
            e.z = rv.x;
            e.w = rv.y;
            sm.rowinfo[threadIdx.x] = e;
        } else {
            // rows past the run: zero residual and phase words, so they add exactly nothing
            sm.rowinfo[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        const unsigned long long pairs = __ballot(my_word & kNewPair);
        wave_lds_order();
        if (j + 1 < nsub) next = fetch_rows<W>(srt, r0, r1, j + 1);
        const int cnt = max(0, min(kWave, we - wb - j * kWave));
        // Blocks of 16 rows, unrolled: row entries through one address register with immediate
        // offsets (an opaque zero keeps the base in a VGPR).
        int zero;
        asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
        const float4 *rsub = rinfo + zero;
        for (int i0 = 0; i0 < cnt; i0 += 16) {
#pragma unroll
            for (int qq = 0; qq < 16; ++qq) {
                const float4 ri = rsub[i0 + qq];
                const float2 rv = make_float2(ri.z, ri.w);
                if ((pairs >> (i0 + qq)) & 1ull) {
                    const int word = __builtin_amdgcn_readlane(my_word, i0 + qq);
                    // close the previous pair and set up the new one
#pragma unroll
                    for (int p = 0; p < kP; ++p) {
                        gr[p] = fmaf(Wpr[p], hr[p], gr[p]);
                        gi_[p] = fmaf(Wpr[p], hi[p], gi_[p]);
                        hr[p] = hi[p] = 0.f;
                    }
                    if (word & kNewG) {
                        const int ga = ant_of_g(g, row_g(word));
#pragma unroll
                        for (int p = 0; p < kP; ++p) {
                            DT dg;
                            float wg;
                            P::geom(sm, ga, vox[p], dg, wg);
                            dG[p] = valid[p] ? dg : DT(0);
                            wG[p] = valid[p] ? wg : 0.f;
                        }
                    }
                    const typename P::LE *lp = lbase + row_l(word) * kBrick;
#pragma unroll
                    for (int p = 0; p < kP; ++p) {
                        const typename P::LE lv = lp[p * kWave];
                        D[p] = P::pair_d(dG[p], lv);
                        Wpr[p] = wG[p] * P::lw(lv);
                    }
                }
#pragma unroll
                for (int p = 0; p < kP; ++p) {
                    const float ph = P::phase(ri, D[p]);
                    const float sn = __builtin_amdgcn_sinf(ph);
                    const float cs = __builtin_amdgcn_cosf(ph);
                    // (cs + j sn)(rv.x + j rv.y)
                    hr[p] = fmaf(cs, rv.x, hr[p]);
                    hr[p] = fmaf(-sn, rv.y, hr[p]);
                    hi[p] = fmaf(cs, rv.y, hi[p]);
                    hi[p] = fmaf(sn, rv.x, hi[p]);
                }
            }
        }
    }
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        gr[p] = fmaf(Wpr[p], hr[p], gr[p]);
        gi_[p] = fmaf(Wpr[p], hi[p], gi_[p]);
    }
    // Combine the waves in a fixed order.
    __syncthreads();
    float2 *red = static_cast<float2 *>(sm.lside);  // W x 256 float2, L-side terms no longer needed
#pragma unroll
    for (int p = 0; p < kP; ++p) red[wave * kBrick + p * kWave + lane] = make_float2(gr[p], gi_[p]);
    __syncthreads();
    const int v = threadIdx.x;
    const int ix = bx * kBX + ((v & 63) & 7), iy = by * kBY + ((v & 63) >> 3), iz = bz * kBZ + (v >> 6);
    if (v < kBrick && ix < g.nx && iy < g.ny && iz < g.nz) {
        float2 acc = red[v];
        for (int w = 1; w < W; ++w) {
            acc.x += red[w * kBrick + v].x;
            acc.y += red[w * kBrick + v].y;
        }
        gpart[(size_t)split * N + ((size_t)iz * g.ny + iy) * g.nx + ix] = acc;
    }
}

template <int MODE, int W>
__global__ __launch_bounds__(W * 64) void k_adj_tile(Geo g, const int4 *__restrict__ srt, int B, int rows_per_wg,
                                                     const float2 *__restrict__ rs, float2 *__restrict__ gpart, int N) {
    extern __shared__ __align__(16) char smem[];
    int tile, split;
    tile_and_split(tile, split);
    const int r0 = split * rows_per_wg;
    adj_tile_body<MODE, W>(g, smem, tile, split, r0, min(B, r0 + rows_per_wg), srt, B, rs, gpart, N);
}

// ------------------------------------------------------------------------------------------
// 5. Column reduction over row splits; optional gradient step and complex soft threshold.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void col_reduce_body(const float2 *__restrict__ gpart, int nsplit, int N,
                                                float2 *__restrict__ g_out, const float2 *s_in, float2 *s_out,
                                                float step, float alpha, int n) {
    if (n >= N) return;
    const float2 gs = split_sum(gpart, nsplit, N, n);
    if (g_out) g_out[n] = gs;
    if (s_out) s_out[n] = prox_step(s_in[n], gs, step, alpha);
}

__global__ __launch_bounds__(256) void k_col_reduce(const float2 *__restrict__ gpart, int nsplit, int N,
                                                    float2 *__restrict__ g_out, float2 *__restrict__ s, float step,
                                                    float alpha) {
    col_reduce_body(gpart, nsplit, N, g_out, s, s, step, alpha, blockIdx.x * blockDim.x + threadIdx.x);
}

// The last step of a solve whose other steps were deferred into the forwards:
// s_out = S_alpha(s_in - step sum_splits gpart); s_in and s_out may be the same array.
__global__ __launch_bounds__(256) void k_col_reduce_to(const float2 *__restrict__ gpart, int nsplit, int N,
                                                       const float2 *s_in, float2 *s_out, float step, float alpha) {
    col_reduce_body(gpart, nsplit, N, nullptr, s_in, s_out, step, alpha, blockIdx.x * blockDim.x + threadIdx.x);
}

// Column reduction of an iteration whose change of magnitudes is recorded (termination rule of
// Sec. V): per voxel the gradient step and soft threshold in place, and per block the fixed-order
// float64 sums of (|s_new| - |s_old|)^2 (part[block]) and |s_old|^2 (part[nb + block]).
constexpr int kChgThreads = 256;
__global__ __launch_bounds__(kChgThreads) void k_col_reduce_change(const float2 *__restrict__ gpart, int nsplit, int N,
                                                                   float2 *__restrict__ s, float step, float alpha,
                                                                   double *__restrict__ part) {
    __shared__ double red[2][kChgThreads];
    const int n = blockIdx.x * kChgThreads + threadIdx.x;
    double d2 = 0.0, o2 = 0.0;
    if (n < N) {
        const float2 old = s[n];
        const float2 nw = prox_step(old, split_sum(gpart, nsplit, N, n), step, alpha);
        s[n] = nw;
        o2 = (double)old.x * old.x + (double)old.y * old.y;
        const double d = sqrt((double)nw.x * nw.x + (double)nw.y * nw.y) - sqrt(o2);
        d2 = d * d;
    }
    red[0][threadIdx.x] = d2;
    red[1][threadIdx.x] = o2;
    __syncthreads();
    for (int w = kChgThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = red[0][0];
        part[gridDim.x + blockIdx.x] = red[1][0];
    }
}

// ------------------------------------------------------------------------------------------
// Ragged batches: many scenes advanced by one launch per phase.  Each scene has a descriptor
// in device memory; tile work is a list of (scene, brick, row range) items ordered longest
// first, walked by persistent work-groups in a fixed round-robin order.
// ------------------------------------------------------------------------------------------
struct SceneDev {
    Geo geo;
    int B, rpw, n_tiles, splits, N;
    const int32_t *rows;  // iteration k uses rows + k * B
    int4 *srt;            // [B]
    const float2 *y;      // [M]
    float2 *s;            // [N]
    float2 *part;         // [n_tiles][B]
    float2 *rs;           // [B]
    float2 *gpart;        // [splits][N]
    float step, alpha;    // eta / B, threshold
};

__device__ __forceinline__ int4 uniform4(int4 v) {
    return make_int4(uniform(v.x), uniform(v.y), uniform(v.z), uniform(v.w));
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scenes(const SceneDev *__restrict__ sc, int iter,
                                                              int *__restrict__ status) {
    extern __shared__ unsigned long long keys[];
    const SceneDev &d = sc[blockIdx.y];
    if ((int)blockIdx.x * kSortChunk >= d.B) return;
    sort_rows_body(d.geo, keys, d.rows + (size_t)iter * d.B, d.B, d.srt, status, blockIdx.x);
}

// At most 128 VGPRs (four waves per SIMD): two work-groups per CU, as the LDS allows.
template <int MODE>
__global__ __launch_bounds__(kThreads, 4) void k_fwd_items(const SceneDev *__restrict__ sc,
                                                           const int4 *__restrict__ items, int n_items) {
    extern __shared__ __align__(16) char smem[];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int4 w = uniform4(items[it]);  // (scene, brick, split, cost)
        const SceneDev &d = sc[w.x];
        const int r0 = w.z * d.rpw;
        fwd_tile_body<MODE>(d.geo, smem, w.y, r0, min(d.B, r0 + d.rpw), d.srt, d.B, d.s, d.part, SStep{}, false);
        __syncthreads();
    }
}

template <int MODE>
__global__ __launch_bounds__(kThreads) void k_adj_items(const SceneDev *__restrict__ sc, const int4 *__restrict__ items,
                                                        int n_items) {
    extern __shared__ __align__(16) char smem[];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int4 w = uniform4(items[it]);
        const SceneDev &d = sc[w.x];
        const int r0 = w.z * d.rpw;
        adj_tile_body<MODE>(d.geo, smem, w.y, w.z, r0, min(d.B, r0 + d.rpw), d.srt, d.B, d.rs, d.gpart, d.N);
        __syncthreads();
    }
}

// blocks[b] = (scene, first row) of 64-row blocks over every scene
__global__ __launch_bounds__(64 * kRedGroups) void k_row_reduce_scenes(const SceneDev *__restrict__ sc,
                                                                      const int2 *__restrict__ blocks, int iter) {
    const int2 b = blocks[blockIdx.x];
    const SceneDev &d = sc[b.x];
    row_reduce_body<64>(d.geo, d.part, d.n_tiles, d.B, d.srt, d.rows + (size_t)iter * d.B, d.y, nullptr, d.rs, b.y);
}

// blocks[b] = (scene, first voxel) of 256-voxel blocks: gradient step and threshold
__global__ __launch_bounds__(256) void k_col_reduce_scenes(const SceneDev *__restrict__ sc,
                                                           const int2 *__restrict__ blocks) {
    const int2 b = blocks[blockIdx.x];
    const SceneDev &d = sc[b.x];
    col_reduce_body(d.gpart, d.splits, d.N, nullptr, d.s, d.s, d.step, d.alpha, b.y + threadIdx.x);
}

// ------------------------------------------------------------------------------------------
// 6. Backward of one unrolled SPGM iteration  s' = S_tau(z),  z = s - (eta/B) g,
//    g = A_B^H (A_B s - y_B).  Gradients use the real-loss convention dL/dRe + j dL/dIm.
// ------------------------------------------------------------------------------------------
constexpr int kVjpThreads = 256;

// Prox VJP per voxel and block partial sums of the two parameter gradients:
//   |z| > tau, u = z/|z|:  zbar = (1 - tau/|z|) sbar + (tau/|z|) u Re(conj(u) sbar),
//                          dL/dtau += -Re(conj(u) sbar);   |z| <= tau: zbar = 0;
//   dL/deta += -(1/B) Re(conj(zbar) g).
__global__ __launch_bounds__(kVjpThreads) void k_prox_vjp(const float2 *__restrict__ s, const float2 *__restrict__ g,
                                                          const float2 *__restrict__ sbar, int N, float step,
                                                          float tau, float inv_b, float2 *__restrict__ zbar,
                                                          double *__restrict__ part) {
    __shared__ double red[2][kVjpThreads];
    const int n = blockIdx.x * kVjpThreads + threadIdx.x;
    double tb = 0.0, eb = 0.0;
    if (n < N) {
        const float2 sv = s[n], gv = g[n], sb = sbar[n];
        const float zx = fmaf(-step, gv.x, sv.x), zy = fmaf(-step, gv.y, sv.y);
        const float r = sqrtf(fmaf(zx, zx, zy * zy));
        float2 zb = make_float2(0.f, 0.f);
        if (r > tau) {
            const float ux = zx / r, uy = zy / r;
            const float re = fmaf(ux, sb.x, uy * sb.y);
            const float c = tau / r;
            zb.x = fmaf(c * re, ux, (1.0f - c) * sb.x);
            zb.y = fmaf(c * re, uy, (1.0f - c) * sb.y);
            tb = -(double)re;
            eb = -(double)inv_b * (double)fmaf(zb.x, gv.x, zb.y * gv.y);
        }
        zbar[n] = zb;
    }
    red[0][threadIdx.x] = tb;
    red[1][threadIdx.x] = eb;
    __syncthreads();
    for (int w = kVjpThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = red[1][0];              // eta
        part[gridDim.x + blockIdx.x] = red[0][0];  // tau
    }
}

// out = zbar - step * h
__global__ __launch_bounds__(256) void k_axpy_out(const float2 *__restrict__ zbar, const float2 *__restrict__ h, int N,
                                                  float step, float2 *__restrict__ out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) {
        const float2 z = zbar[n], hv = h[n];
        out[n] = make_float2(fmaf(-step, hv.x, z.x), fmaf(-step, hv.y, z.y));
    }
}

// Fixed-order sum of the block partials: out[0] = eta gradient, out[1] = tau gradient.
__global__ __launch_bounds__(256) void k_sum_partials(const double *__restrict__ part, int nb,
                                                      double *__restrict__ eta_bar, double *__restrict__ tau_bar) {
    __shared__ double red[2][256];
    double e = 0.0, t = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        e += part[i];
        t += part[nb + i];
    }
    red[0][threadIdx.x] = e;
    red[1][threadIdx.x] = t;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *eta_bar = red[0][0];
        *tau_bar = red[1][0];
    }
}

// ------------------------------------------------------------------------------------------
// Issue-rate probes (roofline denominators).  Every lane runs `iters` rounds of eight
// independent chains of one instruction kind; with 8 work-groups of 256 threads per compute
// unit the chains' latencies are hidden and the launch time measures the issue rate.
//   kind 0: v_fma_f32        kind 1: v_sin_f32        kind 2: v_cos_f32
//   kind 3: the entry body of the tile kernels: phase FMA, sin, cos and four FMAs per chain step
// ------------------------------------------------------------------------------------------
template <int KIND>
__global__ __launch_bounds__(256) void k_probe_rate(float *__restrict__ out, int iters, float seed) {
    float x[8], a[8], b[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        x[j] = seed + 1e-3f * (float)threadIdx.x + 0.125f * (float)j;
        a[j] = 0.f;
        b[j] = 0.f;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (KIND == 0) {
                x[j] = fmaf(x[j], 0.9990234375f, 0.0009765625f);
            } else if (KIND == 1) {
                x[j] = __builtin_amdgcn_sinf(x[j]);
            } else if (KIND == 2) {
                x[j] = __builtin_amdgcn_cosf(x[j]);
            } else {
                const float ph = fmaf(x[j], 0.9990234375f, 0.0009765625f);
                const float sn = __builtin_amdgcn_sinf(ph);
                const float cs = __builtin_amdgcn_cosf(ph);
                a[j] = fmaf(cs, 0.5f, a[j]);
                a[j] = fmaf(sn, 0.25f, a[j]);
                b[j] = fmaf(cs, 0.25f, b[j]);
                b[j] = fmaf(-sn, 0.5f, b[j]);
                x[j] = ph;
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += x[j] + a[j] + b[j];
    if (s == 1234.5f) out[blockIdx.x] = s;  // keeps the chains live; never true in practice
}

#include "spgm_mm.inc"
#include "spgm_sf.inc"
#include "spgm_reg.inc"

// ------------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------------
thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int ok() {
    g_last_error.clear();
    return SPGM_OK;
}

class DeviceGuard {
  public:
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
        if (prev_ != dev) hipSetDevice(dev);
        dev_ = dev;
    }
    ~DeviceGuard() {
        if (prev_ >= 0 && prev_ != dev_) hipSetDevice(prev_);
    }

  private:
    int prev_ = -1, dev_ = 0;
};

// Device address of `scratch` on device `dev` (current), resolved once per device: each GPU
// holds its own copy of the array at its own address.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_addr[kMaxDevices] = {};

char *scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            hipGetLastError();
            return nullptr;
        }
        g_scratch_addr[dev] = static_cast<char *>(ptr);
    }
    return g_scratch_addr[dev];
}

}  // namespace

// Launch shape of a tile kernel: row splits (work-groups per brick) and waves per work-group.
struct TileShape {
    int splits, waves;
};

struct spgm_plan {
    int device = 0;
    int phase_mode = 0;
    int64_t M = 0, N = 0;
    char *scratch = nullptr;  // device address of `scratch` on this plan's device (or nullptr)
    Geo geo{};
    int n_tiles = 0;
    double *d_ant = nullptr;
    double *d_kappa = nullptr;
    float2 *d_q = nullptr;
    int *d_status = nullptr;
    float4 *d_ltab = nullptr;  // precomputed L-side tables (geo.ltab), when they fit
    // workspace, sized for ws_B rows and ws_splits row ranges
    int ws_B = 0;
    int ws_splits = 0;
    int4 *d_srt = nullptr;       // sorted rows of one minibatch
    float2 *d_part = nullptr;    // forward partials [tile][row]
    float2 *d_rs = nullptr;      // scaled residuals, sorted order
    float2 *d_gpart = nullptr;   // adjoint partials [row range][voxel]
    float2 *d_s_alt = nullptr;   // second iterate buffer of a solve [voxel]
    int4 *d_srt_all = nullptr;   // sorted rows of a batch of minibatches (solve)
    float2 *d_vjp = nullptr;     // unrolled backward: g, zbar, h (3 x N) and block partials
    double *d_vjp_part = nullptr;
    // captured solve (spgm_solve_graph): one executable graph and the arguments it was made for
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    struct {
        const int32_t *rows;
        int iters, B;
        const void *y;
        void *s;
        float eta, alpha;
    } graph_key{};
    size_t srt_all_rows = 0;
    size_t lds_bytes = 0;
    // kernel timing instrumentation
    bool timing = false;
    std::vector<hipEvent_t> ev_fwd, ev_adj;  // pairs: [2k] start, [2k+1] stop
    size_t n_fwd = 0, n_adj = 0;
    // waves per work-group of the tile kernels when not tuned (8, or 16 where the brick tables
    // leave room for only one work-group per compute unit)
    int tile_waves = 8;
    // autotuned launch shapes per minibatch size: B -> (forward, adjoint)
    std::map<int, std::pair<TileShape, TileShape>> tuned;
    // autotuned shared-geometry batch shapes per B: {row tiles per wave, bricks per work-group,
    // waves, z slices} of the forward and {row splits, staged rows per round} of the adjoint
    std::map<int, std::array<int, 4>> mm_fwd_tuned;
    std::map<int, std::array<int, 2>> mm_adj_tuned;
    // autotuned structured-minibatch kernels per (nf, nt, nr): items per thread (8 or 16)
    std::map<std::array<int, 3>, int> sf_tuned;
    // default autotuner cache file of this plan (spgm_plan_create_ex; empty: SPGM_TUNE_CACHE)
    std::string tune_cache;
    // minibatches drawn by the seeded generator: device rows (or subsets) of one chunk of
    // iterations and two pinned host staging buffers with their copy-done events
    int32_t *d_gen = nullptr;
    size_t gen_cap = 0;
    int32_t *h_gen[2] = {nullptr, nullptr};
    size_t h_gen_cap = 0;
    hipEvent_t gen_ev[2] = {nullptr, nullptr};
    // shared-geometry batches: packed right-hand sides [tile][z][8][2][64], forward partials
    // [brick run][row][32], packed residuals [row/8][2][64], adjoint partials [split][voxel][32]
    u32x4 *d_mm_s = nullptr;
    float2 *d_gtab = nullptr;  // G-side brick tables of the A-operand-order batched forward
    float2 *d_mm_part = nullptr;
    u32x4 *d_mm_r = nullptr;
    float2 *d_mm_gpart = nullptr;
    size_t mm_part_cap = 0, mm_r_cap = 0, mm_gpart_cap = 0;
    // structured minibatches: measurement index of every row of the current minibatch
    int32_t *d_sf_rows = nullptr;
    size_t sf_rows_cap = 0;
    // TV prox: magnitudes b [voxel] and the dual state w[2], r[2] [voxel] (ping-pong)
    float *d_tv_b = nullptr;
    float4 *d_tv_state = nullptr;
    // solve to the termination rule: iterate at the start of a group of iterations, block
    // partials and per-iteration (change^2, old^2) records, the group's rows for graph replay,
    // and the captured group
    float2 *d_tol_snap = nullptr;
    double *d_tol_part = nullptr;
    double *d_tol_rec = nullptr;
    int32_t *d_tol_rows = nullptr;
    size_t tol_group_cap = 0, tol_rows_cap = 0;
    hipGraph_t tol_graph = nullptr;
    hipGraphExec_t tol_exec = nullptr;
    struct {
        int group, B;
        const void *y;
        void *s;
        float eta, alpha;
    } tol_key{};
};

// A batch of independent scenes (one plan each) advanced together.
constexpr int kBatchRowsPerSplit = 1024;  // default row range of a ragged-batch work item

struct spgm_batch {
    int device = 0;
    int phase_mode = 0;
    std::vector<spgm_plan *> plans;
    hipStream_t cap_stream = nullptr;
    int *d_status = nullptr;
    SceneDev *d_scenes = nullptr;
    size_t scenes_cap = 0;
    int4 *d_items = nullptr;
    size_t items_cap = 0;
    int2 *d_blocks = nullptr;  // row blocks then voxel blocks
    size_t blocks_cap = 0;
    char *d_ws = nullptr;
    size_t ws_cap = 0;
    // launch shape of the tile phases: persistent work-groups (0: fill the chip) and rows per
    // work item
    int max_wg = 0;
    int rows_per_split = kBatchRowsPerSplit;
};

namespace {

constexpr size_t kSolveSortRows = size_t(1) << 25;  // rows sorted ahead per solve batch (512 MiB)
constexpr int kMaxLds = 160 * 1024;                   // LDS per work-group on gfx950

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// Row splits for the tile kernels: the autotuned value for this B if there is one, else enough
// work-groups to cover the chip a few times with at least 64 rows per work-group.
int max_splits(int B) { return std::max(1, (B + 63) / 64); }

int default_splits(const spgm_plan *p, int B) {
    const int want = std::max(1, (4 * 256 + p->n_tiles - 1) / p->n_tiles);
    return std::min(want, max_splits(B));
}

TileShape fwd_shape(const spgm_plan *p, int B) {
    const auto it = p->tuned.find(B);
    return it != p->tuned.end() ? it->second.first : TileShape{default_splits(p, B), p->tile_waves};
}

TileShape adj_shape(const spgm_plan *p, int B) {
    const auto it = p->tuned.find(B);
    return it != p->tuned.end() ? it->second.second : TileShape{default_splits(p, B), p->tile_waves};
}

int fwd_splits(const spgm_plan *p, int B) { return fwd_shape(p, B).splits; }
int adj_splits(const spgm_plan *p, int B) { return adj_shape(p, B).splits; }

// LDS bytes of a tile work-group of `waves` waves: antenna terms, staged rows (16 B row data and
// 8 B row value each), the deferred step's brick iterate, and the L-side table (reused by the
// adjoint for its per-wave column sums).
size_t tile_lds(const Geo &g, int waves) {
    return kAntBytes * (size_t)(g.T + g.R) + (size_t)waves * kWave * (sizeof(float4) + sizeof(float2)) +
           sizeof(float2) * kBrick +
           std::max<size_t>(sizeof(float2) * kBrick * g.nL, sizeof(float2) * kBrick * (size_t)waves);
}

// A captured solve graph holds workspace pointers: drop it whenever the workspace moves.
void drop_graph(spgm_plan *p) {
    if (p->graph_exec) hipGraphExecDestroy(p->graph_exec);
    if (p->graph) hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    if (p->tol_exec) hipGraphExecDestroy(p->tol_exec);
    if (p->tol_graph) hipGraphDestroy(p->tol_graph);
    p->tol_exec = nullptr;
    p->tol_graph = nullptr;
}

int ensure_workspace(spgm_plan *p, int B) {
    const int splits = adj_splits(p, B);
    if (B <= p->ws_B && splits <= p->ws_splits) return SPGM_OK;
    drop_graph(p);
    const int nb = std::max(B, p->ws_B);
    const int ns = std::max(splits, p->ws_splits);
    hipFree(p->d_srt);
    hipFree(p->d_part);
    hipFree(p->d_rs);
    hipFree(p->d_gpart);
    p->d_srt = nullptr;
    p->d_part = nullptr;
    p->d_rs = nullptr;
    p->d_gpart = nullptr;
    p->ws_B = p->ws_splits = 0;
    if (hipMalloc(&p->d_srt, sizeof(int4) * (size_t)nb) != hipSuccess ||
        hipMalloc(&p->d_part, sizeof(float2) * (size_t)nb * p->n_tiles) != hipSuccess ||
        hipMalloc(&p->d_rs, sizeof(float2) * (size_t)nb) != hipSuccess ||
        hipMalloc(&p->d_gpart, sizeof(float2) * (size_t)ns * p->N) != hipSuccess) {
        return fail(SPGM_E_NOMEM, "spgm: workspace allocation failed (B=%d)", nb);
    }
    p->ws_B = nb;
    p->ws_splits = ns;
    return SPGM_OK;
}

int ensure_sorted_batch(spgm_plan *p, size_t rows) {
    if (rows <= p->srt_all_rows) return SPGM_OK;
    drop_graph(p);
    hipFree(p->d_srt_all);
    p->d_srt_all = nullptr;
    p->srt_all_rows = 0;
    if (hipMalloc(&p->d_srt_all, sizeof(int4) * rows) != hipSuccess)
        return fail(SPGM_E_NOMEM, "spgm: sorted-row allocation failed (%zu rows)", rows);
    p->srt_all_rows = rows;
    return SPGM_OK;
}

int launch_check(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SPGM_E_DEVICE, "spgm: %s launch failed: %s", what, hipGetErrorString(e));
    return SPGM_OK;
}

int check_common(spgm_plan *p, const int32_t *rows, int B) {
    if (!p) return fail(SPGM_E_INVALID, "spgm: plan is NULL");
    if (!rows) return fail(SPGM_E_INVALID, "spgm: rows is NULL");
    if (B < 1 || B > kMaxB) return fail(SPGM_E_INVALID, "spgm: B=%d outside [1, %d]", B, kMaxB);
    return SPGM_OK;
}

// Sort `count` consecutive minibatches of B rows each (rows[k*B ...]) into srt[k*B ...].
int run_sort(spgm_plan *p, const int32_t *rows, int B, int count, int4 *srt, hipStream_t st) {
    const int nchunks = (B + kSortChunk - 1) / kSortChunk;
    int p2 = 2;
    while (p2 < std::min(B, kSortChunk)) p2 <<= 1;
    k_sort_rows<<<dim3(nchunks, count), kSortThreads, sizeof(unsigned long long) * p2, st>>>(p->geo, rows, B, srt,
                                                                                           p->d_status);
    return launch_check("sort");
}

// Start/stop events of the next timed launch, growing the pool as needed (nullptr if off).
hipEvent_t *timing_slot(spgm_plan *p, std::vector<hipEvent_t> &pool, size_t &used) {
    if (!p->timing) return nullptr;
    if (2 * used + 2 > pool.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return nullptr;
        if (hipEventCreate(&b) != hipSuccess) {
            hipEventDestroy(a);
            return nullptr;
        }
        pool.push_back(a);
        pool.push_back(b);
    }
    return &pool[2 * used++];
}

// Device workspace of one SPGM step: forward partials [tiles][B], scaled residuals [B] and
// adjoint partials [splits][N] (the plan's own buffers unless a caller brings others).
struct StepWork {
    float2 *part, *rs, *gpart;
};

StepWork plan_work(const spgm_plan *p) { return StepWork{p->d_part, p->d_rs, p->d_gpart}; }

template <int W>
void launch_fwd(const spgm_plan *p, dim3 grid, hipStream_t st, const int4 *srt, int B, int rpw, const float2 *s,
                float2 *part, const SStep &up) {
    const size_t lds = tile_lds(p->geo, W);
    switch (p->phase_mode) {
    case SPGM_PHASE_F64:
        k_fwd_tile<SPGM_PHASE_F64, W><<<grid, W * kWave, lds, st>>>(p->geo, srt, B, rpw, s, part, up);
        break;
    case SPGM_PHASE_NAIVE32:
        k_fwd_tile<SPGM_PHASE_NAIVE32, W><<<grid, W * kWave, lds, st>>>(p->geo, srt, B, rpw, s, part, up);
        break;
    default:
        k_fwd_tile<SPGM_PHASE_COMP32, W><<<grid, W * kWave, lds, st>>>(p->geo, srt, B, rpw, s, part, up);
    }
}

template <int W>
void launch_adj(const spgm_plan *p, dim3 grid, hipStream_t st, const int4 *srt, int B, int rpw, const float2 *rs,
                float2 *gpart) {
    const size_t lds = tile_lds(p->geo, W);
    switch (p->phase_mode) {
    case SPGM_PHASE_F64:
        k_adj_tile<SPGM_PHASE_F64, W><<<grid, W * kWave, lds, st>>>(p->geo, srt, B, rpw, rs, gpart, (int)p->N);
        break;
    case SPGM_PHASE_NAIVE32:
        k_adj_tile<SPGM_PHASE_NAIVE32, W><<<grid, W * kWave, lds, st>>>(p->geo, srt, B, rpw, rs, gpart, (int)p->N);
        break;
    default:
        k_adj_tile<SPGM_PHASE_COMP32, W><<<grid, W * kWave, lds, st>>>(p->geo, srt, B, rpw, rs, gpart, (int)p->N);
    }
}

int run_forward_partials(spgm_plan *p, const int4 *srt, const float2 *s, int B, hipStream_t st,
                         const SStep &up = SStep{}, float2 *part = nullptr) {
    if (!part) part = p->d_part;
    const TileShape sh = fwd_shape(p, B);
    const int rpw = (B + sh.splits - 1) / sh.splits;
    hipEvent_t *ev = timing_slot(p, p->ev_fwd, p->n_fwd);
    if (ev) hipEventRecord(ev[0], st);
    const dim3 grid(p->n_tiles, sh.splits);
    if (sh.waves == 16)
        launch_fwd<16>(p, grid, st, srt, B, rpw, s, part, up);
    else
        launch_fwd<8>(p, grid, st, srt, B, rpw, s, part, up);
    if (ev) hipEventRecord(ev[1], st);
    return launch_check("forward");
}

int run_adjoint_partials(spgm_plan *p, const int4 *srt, int B, hipStream_t st, const float2 *rs = nullptr,
                         float2 *gpart = nullptr) {
    if (!rs) rs = p->d_rs;
    if (!gpart) gpart = p->d_gpart;
    const TileShape sh = adj_shape(p, B);
    const int rpw = (B + sh.splits - 1) / sh.splits;
    hipEvent_t *ev = timing_slot(p, p->ev_adj, p->n_adj);
    if (ev) hipEventRecord(ev[0], st);
    const dim3 grid(p->n_tiles, sh.splits);
    if (sh.waves == 16)
        launch_adj<16>(p, grid, st, srt, B, rpw, rs, gpart);
    else
        launch_adj<8>(p, grid, st, srt, B, rpw, rs, gpart);
    if (ev) hipEventRecord(ev[1], st);
    return launch_check("adjoint");
}

int run_row_reduce(spgm_plan *p, const int4 *srt, const int32_t *rows, int B, const float2 *y, float2 *out_user,
                   float2 *out_scaled, hipStream_t st, const float2 *part = nullptr) {
    if (!part) part = p->d_part;
    k_row_reduce<<<(B + kRedRows - 1) / kRedRows, kRedRows * kRedGroups, 0, st>>>(p->geo, part, p->n_tiles, B, srt,
                                                                                  rows, y, out_user, out_scaled);
    return launch_check("row reduce");
}

// One SPGM iteration on already sorted rows, in workspace w.
int step_sorted(spgm_plan *p, const int4 *srt, const int32_t *rows, int B, const float2 *y, float2 *s, float eta,
                float alpha, hipStream_t st, const StepWork &w) {
    int rc;
    if ((rc = run_forward_partials(p, srt, s, B, st, SStep{}, w.part))) return rc;
    if ((rc = run_row_reduce(p, srt, rows, B, y, nullptr, w.rs, st, w.part))) return rc;
    if ((rc = run_adjoint_partials(p, srt, B, st, w.rs, w.gpart))) return rc;
    k_col_reduce<<<(int)((p->N + 255) / 256), 256, 0, st>>>(w.gpart, adj_splits(p, B), (int)p->N, nullptr, s,
                                                             eta / (float)B, alpha);
    return launch_check("column reduce");
}

// ---------------------------------------------------------------- other regularisers
constexpr int kMaxTVIters = 100000;

int check_reg(const spgm_regularizer *reg) {
    if (!reg) return fail(SPGM_E_INVALID, "spgm: regularizer is NULL");
    if (reg->kind < SPGM_REG_L1 || reg->kind > SPGM_REG_TV_MAGNITUDE)
        return fail(SPGM_E_INVALID, "spgm: unknown regularizer kind %d", (int)reg->kind);
    if (reg->kind == SPGM_REG_ELASTIC_NET && !(std::isfinite(reg->mu) && reg->mu >= 0))
        return fail(SPGM_E_INVALID, "spgm: elastic-net mu must be finite and >= 0");
    if (reg->kind == SPGM_REG_TV_MAGNITUDE && (reg->tv_iters < 0 || reg->tv_iters > kMaxTVIters))
        return fail(SPGM_E_INVALID, "spgm: tv_iters must be in [0, %d]", kMaxTVIters);
    return SPGM_OK;
}

int ensure_tv(spgm_plan *p) {
    if (p->d_tv_b) return SPGM_OK;
    if (hipMalloc(&p->d_tv_b, sizeof(float) * (size_t)p->N) != hipSuccess) {
        p->d_tv_b = nullptr;
        return fail(SPGM_E_NOMEM, "spgm: TV workspace allocation failed");
    }
    if (hipMalloc(&p->d_tv_state, sizeof(float4) * 4 * (size_t)p->N) != hipSuccess) {
        hipFree(p->d_tv_b);
        p->d_tv_b = nullptr;
        p->d_tv_state = nullptr;
        return fail(SPGM_E_NOMEM, "spgm: TV workspace allocation failed");
    }
    return SPGM_OK;
}

float elastic_scale(float alpha, float mu) { return (float)(1.0 / (1.0 + (double)alpha * (double)mu)); }

// TV prox of v in place (workspace allocated): `iters` dual iterations and the final primal point.
int run_tv_prox(spgm_plan *p, float2 *v, float alpha, int iters, hipStream_t st) {
    if (alpha == 0.f || iters == 0) return SPGM_OK;
    const TVGrid g{p->geo.nx, p->geo.ny, p->geo.nz, (int)p->N, p->geo.nx * p->geo.ny};
    const int nb = (g.N + kRegThreads - 1) / kRegThreads;
    float4 *w[2] = {p->d_tv_state, p->d_tv_state + p->N};
    float4 *r[2] = {p->d_tv_state + 2 * p->N, p->d_tv_state + 3 * p->N};
    const float inv12a = (float)(1.0 / (12.0 * (double)alpha));
    double t = 1.0;
    int rc;
    for (int k = 1; k <= iters; ++k) {
        const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
        const float beta = (float)((t - 1.0) / tn);
        t = tn;
        if (k == 1)
            k_tv_iter<true><<<nb, kRegThreads, 0, st>>>(g, v, p->d_tv_b, nullptr, nullptr, w[1], r[1], alpha, inv12a,
                                                        0.f);
        else
            k_tv_iter<false><<<nb, kRegThreads, 0, st>>>(g, v, p->d_tv_b, r[(k - 1) & 1], w[(k - 1) & 1], w[k & 1],
                                                         r[k & 1], alpha, inv12a, beta);
        if ((rc = launch_check("tv dual iteration"))) return rc;
    }
    k_tv_finish<<<nb, kRegThreads, 0, st>>>(g, v, p->d_tv_b, w[iters & 1], alpha);
    return launch_check("tv finish");
}

// One iteration on already sorted rows with the prox of `reg` (validated, workspace allocated).
int step_sorted_reg(spgm_plan *p, const int4 *srt, const int32_t *rows, int B, const float2 *y, float2 *s, float eta,
                    float alpha, const spgm_regularizer &reg, hipStream_t st) {
    if (reg.kind == SPGM_REG_L1) return step_sorted(p, srt, rows, B, y, s, eta, alpha, st, plan_work(p));
    int rc;
    if ((rc = run_forward_partials(p, srt, s, B, st))) return rc;
    if ((rc = run_row_reduce(p, srt, rows, B, y, nullptr, p->d_rs, st))) return rc;
    if ((rc = run_adjoint_partials(p, srt, B, st))) return rc;
    const int nb = (int)((p->N + kRegThreads - 1) / kRegThreads);
    if (reg.kind == SPGM_REG_ELASTIC_NET) {
        k_col_reduce_elastic<<<nb, kRegThreads, 0, st>>>(p->d_gpart, adj_splits(p, B), (int)p->N, s, eta / (float)B,
                                                         alpha, elastic_scale(alpha, reg.mu));
        return launch_check("column reduce (elastic net)");
    }
    // gradient step only (a zero threshold leaves every value unchanged), then the TV prox
    k_col_reduce<<<(int)((p->N + 255) / 256), 256, 0, st>>>(p->d_gpart, adj_splits(p, B), (int)p->N, nullptr, s,
                                                             eta / (float)B, 0.f);
    if ((rc = launch_check("column reduce"))) return rc;
    return run_tv_prox(p, s, alpha, reg.tv_iters, st);
}

int ensure_vjp(spgm_plan *p) {
    if (p->d_vjp) return SPGM_OK;
    const int nb = (int)((p->N + kVjpThreads - 1) / kVjpThreads);
    if (hipMalloc(&p->d_vjp, sizeof(float2) * 3 * (size_t)p->N) != hipSuccess ||
        hipMalloc(&p->d_vjp_part, sizeof(double) * 2 * (size_t)nb) != hipSuccess)
        return fail(SPGM_E_NOMEM, "spgm: backward workspace allocation failed");
    return SPGM_OK;
}


// ---------------------------------------------------------------- shared-geometry batches
template <typename T> int grow_buf(T *&ptr, size_t &cap, size_t need) {
    if (need <= cap) return SPGM_OK;
    hipFree(ptr);
    ptr = nullptr;
    cap = 0;
    if (hipMalloc(&ptr, sizeof(T) * need) != hipSuccess)
        return fail(SPGM_E_NOMEM, "spgm: batched workspace allocation failed (%zu bytes)", sizeof(T) * need);
    cap = need;
    return SPGM_OK;
}

// Forward launch shape: rows per wave 32 nrt (nrt = 1..4), work-groups of 32 nrt rows per wave,
// bricks grouped into runs of bpw (each run leaves one partial sum per row, right-hand side and
// z range).  The A-operand-order form (k_mm_fwd_rows) needs the plan's L-side table and both
// brick tables in LDS; it runs 8 waves over the whole brick or 4 waves over two z slices (two
// work-groups per compute unit).  k_mm_fwd (entry tile through LDS) runs 8 waves per brick.
struct MMFwdCfg {
    int nrt = 1, rows_wg = 0, n_rb = 0, bpw = 1, n_super = 0;
    int waves = kWaves, zs = kBZ;  // waves per work-group, z slices per work-group
    bool rows_form = false;        // k_mm_fwd_rows (entries in A-operand order) instead of k_mm_fwd
    size_t lds = 0;
    int n_slots() const { return n_super * (kBZ / zs); }
};

// Bricks per work-group that launch about one round of work-groups (8 waves per compute unit).
int mm_default_bpw(const spgm_plan *p, int n_rb, int waves, int zs) {
    const int target = 256 * (kWaves / waves);
    return std::max(1, (p->n_tiles * n_rb * (kBZ / zs) + target - 1) / target);
}

// The forward shape for explicit choices (bpw = 0: the default for the rest); false if it does
// not fit this plan.
bool mm_fwd_shape(const spgm_plan *p, int B, int nrt, int bpw, int waves, int zs, MMFwdCfg &c) {
    const int A = p->geo.T + p->geo.R, nG = p->geo.nG, nL = p->geo.nL;
    if (nrt < 1 || nrt > 4 || bpw < 0) return false;
    c = MMFwdCfg{};
    const bool rows_ok = p->d_ltab && p->geo.ltab_mode == SPGM_PHASE_COMP32 &&
                         ((waves == 8 && zs == 4) || (waves == 4 && zs == 2));
    if (rows_ok && mm_fwd_rows_lds(nrt, A, nG, nL, waves, zs) <= (size_t)kMaxLds) {
        c.rows_form = true;
        c.lds = mm_fwd_rows_lds(nrt, A, nG, nL, waves, zs);
    } else if (waves == kWaves && zs == kBZ && mm_fwd_lds(nrt, A, nL) <= (size_t)kMaxLds) {
        c.lds = mm_fwd_lds(nrt, A, nL);
    } else {
        return false;
    }
    c.nrt = nrt;
    c.waves = waves;
    c.zs = zs;
    c.rows_wg = waves * kMMRows * nrt;
    c.n_rb = (B + c.rows_wg - 1) / c.rows_wg;
    c.bpw = std::min(p->n_tiles, bpw > 0 ? bpw : mm_default_bpw(p, c.n_rb, waves, zs));
    c.n_super = (p->n_tiles + c.bpw - 1) / c.bpw;
    return true;
}

// The autotuned forward shape for this B if there is one, else 8 waves over whole bricks with as
// many row tiles per wave (up to 4, one per 256 rows of the minibatch) as LDS allows.
MMFwdCfg mm_fwd_cfg(const spgm_plan *p, int B) {
    MMFwdCfg c;
    const auto it = p->mm_fwd_tuned.find(B);
    if (it != p->mm_fwd_tuned.end()) {
        const auto &v = it->second;
        if (mm_fwd_shape(p, B, v[0], v[1], v[2], v[3], c)) return c;
    }
    const int want = std::min(4, std::max(1, (B + kWaves * kMMRows - 1) / (kWaves * kMMRows)));
    for (int nrt = want; nrt >= 1; --nrt)
        if (mm_fwd_shape(p, B, nrt, 0, kWaves, kBZ, c)) return c;
    c.lds = (size_t)kMaxLds + 1;  // nothing fits: mm_check refuses
    return c;
}

// Adjoint launch shape: one work-group per (brick, row range); row ranges are multiples of 512
// rows (four row groups), by default split only when there are fewer than 256 bricks.  Each
// round stages `stage` rows per group (a multiple of kMMStage): by default the whole group when
// LDS holds it beside the L-side table, else the largest multiple that fits.
struct MMAdjCfg {
    int splits = 1, rpw = 0, stage = 0;
    size_t lds = 0;
};

int mm_default_adj_splits(const spgm_plan *p, int B) {
    const int unit = kMMGroups * 128;
    const int splits = std::max(1, (256 + p->n_tiles - 1) / p->n_tiles);
    return std::min(splits, (B + unit - 1) / unit);
}

// The adjoint shape for explicit choices (stage = 0: as large as useful and LDS allows); false if
// it does not fit this plan.
bool mm_adj_shape(const spgm_plan *p, int B, int splits, int stage, MMAdjCfg &c) {
    const int unit = kMMGroups * 128;
    if (splits < 1 || stage < 0 || stage % kMMStage != 0) return false;
    c = MMAdjCfg{};
    c.rpw = ((B + splits - 1) / splits + unit - 1) / unit * unit;
    c.splits = (B + c.rpw - 1) / c.rpw;
    const int A = p->geo.T + p->geo.R;
    const int per = (std::min(c.rpw, B) + kMMGroups - 1) / kMMGroups;
    const int full = (per + kMMStage - 1) / kMMStage * kMMStage;
    if (stage == 0) {
        const size_t fixed = mm_adj_lds(A, p->geo.nL, 0);
        const int cap = fixed >= (size_t)kMaxLds
                            ? 0
                            : (int)((kMaxLds - fixed) / (sizeof(float4) * kMMGroups)) / kMMStage * kMMStage;
        stage = std::max(kMMStage, std::min(cap, full));
    }
    c.stage = std::min(stage, std::max(kMMStage, full));
    c.lds = mm_adj_lds(A, p->geo.nL, c.stage);
    return c.lds <= (size_t)kMaxLds;
}

MMAdjCfg mm_adj_cfg(const spgm_plan *p, int B) {
    MMAdjCfg c;
    const auto it = p->mm_adj_tuned.find(B);
    if (it != p->mm_adj_tuned.end() && mm_adj_shape(p, B, it->second[0], it->second[1], c)) return c;
    if (!mm_adj_shape(p, B, mm_default_adj_splits(p, B), 0, c)) c.lds = (size_t)kMaxLds + 1;
    return c;
}

int mm_check(spgm_plan *p, const int32_t *rows, int B, int K, int prec, const char *who) {
    int rc;
    if ((rc = check_common(p, rows, B))) return rc;
    if (K < 1) return fail(SPGM_E_INVALID, "%s: K must be >= 1", who);
    if (prec != SPGM_MM_BF16 && prec != SPGM_MM_FP16) return fail(SPGM_E_INVALID, "%s: unknown precision %d", who, prec);
    if (p->phase_mode != SPGM_PHASE_COMP32)
        return fail(SPGM_E_UNSUPPORTED, "%s: needs a plan created with SPGM_PHASE_COMP32", who);
    if (mm_fwd_cfg(p, B).lds > (size_t)kMaxLds || mm_adj_cfg(p, B).lds > (size_t)kMaxLds)
        return fail(SPGM_E_UNSUPPORTED, "%s: brick tables exceed LDS (smaller antenna array too large)", who);
    return SPGM_OK;
}

int ensure_mm(spgm_plan *p, int B) {
    int rc;
    if ((rc = ensure_workspace(p, B))) return rc;  // sorted rows
    const MMFwdCfg fc = mm_fwd_cfg(p, B);
    const MMAdjCfg ac = mm_adj_cfg(p, B);
    if (!p->d_mm_s && hipMalloc(&p->d_mm_s, sizeof(u32x4) * kMMSlice * kBZ * (size_t)p->n_tiles) != hipSuccess)
        return fail(SPGM_E_NOMEM, "spgm: batched workspace allocation failed");
    if (fc.rows_form && !p->d_gtab) {
        // G-side brick tables for the A-operand-order forward, formed once per plan
        if (hipMalloc(&p->d_gtab, sizeof(float2) * kBrick * (size_t)p->geo.nG * p->n_tiles) != hipSuccess) {
            p->d_gtab = nullptr;
            return fail(SPGM_E_NOMEM, "spgm: batched G-side table allocation failed");
        }
        hipFuncSetAttribute((const void *)k_build_gtab, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p->lds_bytes);
        k_build_gtab<<<p->n_tiles, kThreads, p->lds_bytes>>>(p->geo, p->d_gtab);
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
            hipFree(p->d_gtab);
    hipFree(p->d_gen);
    for (int i = 0; i < 2; ++i) {
        if (p->h_gen[i]) hipHostFree(p->h_gen[i]);
        if (p->gen_ev[i]) hipEventDestroy(p->gen_ev[i]);
    }
            p->d_gtab = nullptr;
            return fail(SPGM_E_DEVICE, "spgm: batched G-side table build failed");
        }
    }
    if ((rc = grow_buf(p->d_mm_part, p->mm_part_cap, (size_t)fc.n_slots() * B * kMMCols))) return rc;
    if ((rc = grow_buf(p->d_mm_r, p->mm_r_cap, (size_t)((B + 7) / 8) * 2 * 64))) return rc;
    if (ac.splits > 1 && (rc = grow_buf(p->d_mm_gpart, p->mm_gpart_cap, (size_t)ac.splits * p->N * kMMCols)))
        return rc;  // one split: the adjoint writes its outputs itself
    return SPGM_OK;
}

// Forward pass of right-hand sides k0 .. k0+K-1 of S ([N][ld]) into the plan's partials.
// pack = false: the packed operand already holds these right-hand sides (written by the previous
// step's adjoint).
template <int PREC>
int mm_forward_pass(spgm_plan *p, const MMFwdCfg &fc, const int4 *srt, int B, const float2 *S, int ld, int k0,
                    int K, hipStream_t st, bool pack = true) {
    int rc;
    if (pack) {
        const size_t nth = (size_t)p->n_tiles * 2048;
        k_mm_pack_s<PREC><<<(unsigned)((nth + 255) / 256), 256, 0, st>>>(p->geo, S, ld, k0, K, p->n_tiles, p->d_mm_s);
        if ((rc = launch_check("batched pack"))) return rc;
    }
    hipEvent_t *ev = timing_slot(p, p->ev_fwd, p->n_fwd);
    if (ev) hipEventRecord(ev[0], st);
    if (fc.rows_form) {
        const dim3 grid(fc.n_super, fc.n_rb, kBZ / fc.zs);
        const int nth = fc.waves * kWave;
        const float4 *gt = reinterpret_cast<const float4 *>(p->d_gtab);
        switch (fc.nrt) {
        case 1:
            k_mm_fwd_rows<PREC, 1><<<grid, nth, fc.lds, st>>>(p->geo, srt, B, fc.bpw, p->n_tiles, fc.zs, gt, p->d_mm_s,
                                                             p->d_mm_part);
            break;
        case 2:
            k_mm_fwd_rows<PREC, 2><<<grid, nth, fc.lds, st>>>(p->geo, srt, B, fc.bpw, p->n_tiles, fc.zs, gt, p->d_mm_s,
                                                             p->d_mm_part);
            break;
        case 3:
            k_mm_fwd_rows<PREC, 3><<<grid, nth, fc.lds, st>>>(p->geo, srt, B, fc.bpw, p->n_tiles, fc.zs, gt, p->d_mm_s,
                                                             p->d_mm_part);
            break;
        default:
            k_mm_fwd_rows<PREC, 4><<<grid, nth, fc.lds, st>>>(p->geo, srt, B, fc.bpw, p->n_tiles, fc.zs, gt, p->d_mm_s,
                                                             p->d_mm_part);
        }
        if (ev) hipEventRecord(ev[1], st);
        return launch_check("batched forward");
    }
    const dim3 grid(fc.n_super, fc.n_rb);
    switch (fc.nrt) {
    case 1:
        k_mm_fwd<PREC, 1><<<grid, kThreads, fc.lds, st>>>(p->geo, srt, B, fc.bpw, p->n_tiles, p->d_mm_s, p->d_mm_part);
        break;
    case 2:
        k_mm_fwd<PREC, 2><<<grid, kThreads, fc.lds, st>>>(p->geo, srt, B, fc.bpw, p->n_tiles, p->d_mm_s, p->d_mm_part);
        break;
    case 3:
        k_mm_fwd<PREC, 3><<<grid, kThreads, fc.lds, st>>>(p->geo, srt, B, fc.bpw, p->n_tiles, p->d_mm_s, p->d_mm_part);
        break;
    default:
        k_mm_fwd<PREC, 4><<<grid, kThreads, fc.lds, st>>>(p->geo, srt, B, fc.bpw, p->n_tiles, p->d_mm_s, p->d_mm_part);
    }
    if (ev) hipEventRecord(ev[1], st);
    return launch_check("batched forward");
}

template <int PREC>
int mm_row_reduce(spgm_plan *p, const MMFwdCfg &fc, const int4 *srt, const int32_t *rows, int B, const float2 *y,
                  int ldy, int k0, int K, float2 *out, int ldo, bool want_r, hipStream_t st) {
    const int quads = ((B + 7) & ~7) / 4;
    k_mm_row_reduce<PREC><<<(quads + 7) / 8, 256, 0, st>>>(p->geo, p->d_mm_part, fc.n_slots(), B, srt, rows, y, ldy, k0,
                                                            K, out, ldo, want_r ? p->d_mm_r : nullptr);
    return launch_check("batched row reduce");
}

// Adjoint pass and its outputs: with one row split the adjoint kernel writes g and the proximal
// update itself (and the next packed operand when s2 is set); otherwise it leaves per-split
// partials that k_mm_col_reduce sums in a fixed order.
template <int PREC>
int mm_adjoint_pass(spgm_plan *p, const MMAdjCfg &ac, const int4 *srt, int B, const MMAdjOut &out, hipStream_t st) {
    hipEvent_t *ev = timing_slot(p, p->ev_adj, p->n_adj);
    if (ev) hipEventRecord(ev[0], st);
    const bool fused = ac.splits == 1;
    MMAdjOut o = out;
    if (!fused) o.s2 = nullptr;
    k_mm_adj<PREC><<<dim3(p->n_tiles, ac.splits), kThreads, ac.lds, st>>>(
        p->geo, srt, B, ac.rpw, ac.stage, p->d_mm_r, fused ? nullptr : p->d_mm_gpart, (int)p->N, o);
    if (ev) hipEventRecord(ev[1], st);
    int rc;
    if ((rc = launch_check("batched adjoint")) || fused) return rc;
    const size_t nth = (size_t)p->N * kMMCols;
    k_mm_col_reduce<<<(unsigned)((nth + 255) / 256), 256, 0, st>>>(p->d_mm_gpart, ac.splits, (int)p->N, out.k0,
                                                                   out.K, out.ld, out.g, out.s, out.step, out.alpha);
    return launch_check("batched column reduce");
}

// Y = A_B S over passes of 32 right-hand sides.
template <int PREC>
int mm_forward(spgm_plan *p, const int4 *srt, const int32_t *rows, int B, int K, const float2 *S, float2 *Y,
               hipStream_t st) {
    const MMFwdCfg fc = mm_fwd_cfg(p, B);
    int rc;
    for (int k0 = 0; k0 < K; k0 += kMMCols) {
        const int kc = std::min(kMMCols, K - k0);
        if ((rc = mm_forward_pass<PREC>(p, fc, srt, B, S, K, k0, kc, st))) return rc;
        if ((rc = mm_row_reduce<PREC>(p, fc, srt, rows, B, nullptr, 0, k0, kc, Y, K, false, st))) return rc;
    }
    return SPGM_OK;
}

// G = A_B^H R over passes of 32 right-hand sides.
template <int PREC>
int mm_adjoint(spgm_plan *p, const int4 *srt, int B, int K, const float2 *R, float2 *G, hipStream_t st) {
    const MMAdjCfg ac = mm_adj_cfg(p, B);
    int rc;
    for (int k0 = 0; k0 < K; k0 += kMMCols) {
        const int kc = std::min(kMMCols, K - k0);
        const int quads = ((B + 7) & ~7) / 4;
        k_mm_pack_r<PREC><<<(quads + 7) / 8, 256, 0, st>>>(p->geo, srt, B, R, K, k0, kc, p->d_mm_r);
        if ((rc = launch_check("batched pack"))) return rc;
        const MMAdjOut out{k0, kc, K, G, nullptr, 0.f, 0.f, nullptr};
        if ((rc = mm_adjoint_pass<PREC>(p, ac, srt, B, out, st))) return rc;
    }
    return SPGM_OK;
}

// One batched SPGM iteration on sorted rows.  With K <= 32 and an unsplit adjoint the step can
// leave the packed operand of its result for the next step (s2_out) and take it from the
// previous one (packed_in).
template <int PREC>
int mm_step(spgm_plan *p, const int4 *srt, const int32_t *rows, int B, int K, const float2 *Ym, float2 *S, float eta,
            float alpha, hipStream_t st, bool packed_in = false, bool s2_out = false) {
    const MMFwdCfg fc = mm_fwd_cfg(p, B);
    const MMAdjCfg ac = mm_adj_cfg(p, B);
    int rc;
    for (int k0 = 0; k0 < K; k0 += kMMCols) {
        const int kc = std::min(kMMCols, K - k0);
        if ((rc = mm_forward_pass<PREC>(p, fc, srt, B, S, K, k0, kc, st, !packed_in))) return rc;
        if ((rc = mm_row_reduce<PREC>(p, fc, srt, rows, B, Ym, K, k0, kc, nullptr, 0, true, st))) return rc;
        const MMAdjOut out{k0, kc, K, nullptr, S, eta / (float)B, alpha, s2_out ? p->d_mm_s : nullptr};
        if ((rc = mm_adjoint_pass<PREC>(p, ac, srt, B, out, st))) return rc;
    }
    return SPGM_OK;
}

// Whether consecutive steps can hand the packed operand on (one pass, unsplit adjoint).
bool mm_chain_ok(const spgm_plan *p, int B, int K) { return K <= kMMCols && mm_adj_cfg(p, B).splits == 1; }

int mm_step_any(spgm_plan *p, int prec, const int4 *srt, const int32_t *rows, int B, int K, const float2 *Ym,
                float2 *S, float eta, float alpha, hipStream_t st, bool packed_in = false, bool s2_out = false) {
    return prec == SPGM_MM_FP16
               ? mm_step<SPGM_MM_FP16>(p, srt, rows, B, K, Ym, S, eta, alpha, st, packed_in, s2_out)
               : mm_step<SPGM_MM_BF16>(p, srt, rows, B, K, Ym, S, eta, alpha, st, packed_in, s2_out);
}

// ---------------------------------------------------------------- structured minibatches
struct SFArgs {
    const int32_t *fi, *ti, *ri;
    int nf, nt, nr, B;
};

int sf_check(spgm_plan *p, const SFArgs &a, const char *who) {
    if (!p) return fail(SPGM_E_INVALID, "%s: plan is NULL", who);
    if (!a.fi || !a.ti || !a.ri) return fail(SPGM_E_INVALID, "%s: index arrays must be non-NULL", who);
    if (a.nf < 1 || a.nf > 65535 || a.nt < 1 || a.nr < 1 || a.nt > kSFMax || a.nr > kSFMax)
        return fail(SPGM_E_INVALID, "%s: need 1 <= nf <= 65535 and 1 <= nt, nr <= %d", who, kSFMax);
    if ((int64_t)a.nf * a.nt * a.nr > kMaxB) return fail(SPGM_E_INVALID, "%s: nf*nt*nr exceeds %d", who, kMaxB);
    if (p->phase_mode != SPGM_PHASE_COMP32)
        return fail(SPGM_E_UNSUPPORTED, "%s: needs a plan created with SPGM_PHASE_COMP32", who);
    if (sf_lds_bytes(p->geo.T + p->geo.R) > (size_t)kMaxLds)
        return fail(SPGM_E_UNSUPPORTED, "%s: antenna tables exceed LDS", who);
    return SPGM_OK;
}

// Workspace and the row table of a structured minibatch (sorted-row format, natural order).
int sf_prepare(spgm_plan *p, const SFArgs &a, hipStream_t st) {
    int rc;
    if ((rc = ensure_workspace(p, a.B))) return rc;
    if ((rc = grow_buf(p->d_sf_rows, p->sf_rows_cap, (size_t)a.B))) return rc;
    k_sf_rows<<<(a.B + 255) / 256, 256, 0, st>>>(p->geo, a.fi, a.nf, a.ti, a.nt, a.ri, a.nr, p->d_srt, p->d_sf_rows,
                                                  p->d_status);
    return launch_check("structured rows");
}

// Subsets of at most 32 antennas in all, at most 16 of them transmitters, may take the kernels'
// small-register instances (8 items per thread); they do unless the autotuner chose the general
// ones (16 items) for this (nf, nt, nr).
bool sf_small_ok(const SFArgs &a) { return a.nt + a.nr <= 32 && a.nt <= 16; }

bool sf_small(const spgm_plan *p, const SFArgs &a) {
    if (!sf_small_ok(a)) return false;
    const auto it = p->sf_tuned.find({a.nf, a.nt, a.nr});
    return it == p->sf_tuned.end() || it->second == kSFItemsSmall;
}

int sf_forward_partials(spgm_plan *p, const SFArgs &a, const float2 *s, hipStream_t st) {
    hipEvent_t *ev = timing_slot(p, p->ev_fwd, p->n_fwd);
    if (ev) hipEventRecord(ev[0], st);
    const size_t lds = sf_lds_bytes(p->geo.T + p->geo.R);
    if (sf_small(p, a))
        k_sf_fwd<kSFItemsSmall><<<p->n_tiles, kThreads, lds, st>>>(p->geo, a.fi, a.nf, a.ti, a.nt, a.ri, a.nr, s,
                                                                   p->d_part, a.B);
    else
        k_sf_fwd<kSFItems><<<p->n_tiles, kThreads, lds, st>>>(p->geo, a.fi, a.nf, a.ti, a.nt, a.ri, a.nr, s,
                                                              p->d_part, a.B);
    if (ev) hipEventRecord(ev[1], st);
    return launch_check("structured forward");
}

// Adjoint of the scaled residuals in p->d_rs into p->d_gpart[0].
int sf_adjoint_partials(spgm_plan *p, const SFArgs &a, hipStream_t st) {
    hipEvent_t *ev = timing_slot(p, p->ev_adj, p->n_adj);
    if (ev) hipEventRecord(ev[0], st);
    const size_t lds = sf_lds_bytes(p->geo.T + p->geo.R);
    if (sf_small(p, a))
        k_sf_adj<kSFItemsSmall, 1><<<p->n_tiles, kThreads, lds, st>>>(p->geo, a.fi, a.nf, a.ti, a.nt, a.ri, a.nr,
                                                                      p->d_rs, p->d_gpart, (int)p->N);
    else
        k_sf_adj<kSFItems, 2><<<p->n_tiles, kThreads, lds, st>>>(p->geo, a.fi, a.nf, a.ti, a.nt, a.ri, a.nr, p->d_rs,
                                                                 p->d_gpart, (int)p->N);
    if (ev) hipEventRecord(ev[1], st);
    return launch_check("structured adjoint");
}

int sf_step(spgm_plan *p, const SFArgs &a, const float2 *y, float2 *s, float eta, float alpha, hipStream_t st) {
    int rc;
    if ((rc = sf_prepare(p, a, st))) return rc;
    if ((rc = sf_forward_partials(p, a, s, st))) return rc;
    if ((rc = run_row_reduce(p, p->d_srt, p->d_sf_rows, a.B, y, nullptr, p->d_rs, st))) return rc;
    if ((rc = sf_adjoint_partials(p, a, st))) return rc;
    k_col_reduce<<<(int)((p->N + 255) / 256), 256, 0, st>>>(p->d_gpart, 1, (int)p->N, nullptr, s, eta / (float)a.B,
                                                             alpha);
    return launch_check("column reduce");
}

}  // namespace

extern "C" {

const char *spgm_last_error(void) { return g_last_error.c_str(); }

// L-side tables of every brick (geometry only), formed once per plan with the same code the tile
// kernels would run and then copied by them instead of formed by every work-group.  Skipped
// (the kernels form the tables themselves) when they would exceed kMaxLtabBytes or cannot be
// allocated; the results are the same either way, bit for bit.
static constexpr size_t kMaxLtabBytes = size_t(8) << 30;

static void build_ltab(spgm_plan *p) {
    Geo &g = p->geo;
    const size_t bytes = sizeof(float2) * kBrick * (size_t)g.nL * (size_t)p->n_tiles;
    if (bytes > kMaxLtabBytes || hipMalloc(&p->d_ltab, bytes) != hipSuccess) {
        p->d_ltab = nullptr;
        hipGetLastError();
        return;
    }
    const void *fn = p->phase_mode == SPGM_PHASE_F64       ? (const void *)k_build_ltab<SPGM_PHASE_F64>
                     : p->phase_mode == SPGM_PHASE_NAIVE32 ? (const void *)k_build_ltab<SPGM_PHASE_NAIVE32>
                                                           : (const void *)k_build_ltab<SPGM_PHASE_COMP32>;
    hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p->lds_bytes);
    switch (p->phase_mode) {
    case SPGM_PHASE_F64:
        k_build_ltab<SPGM_PHASE_F64><<<p->n_tiles, kThreads, p->lds_bytes>>>(g, p->d_ltab);
        break;
    case SPGM_PHASE_NAIVE32:
        k_build_ltab<SPGM_PHASE_NAIVE32><<<p->n_tiles, kThreads, p->lds_bytes>>>(g, p->d_ltab);
        break;
    default:
        k_build_ltab<SPGM_PHASE_COMP32><<<p->n_tiles, kThreads, p->lds_bytes>>>(g, p->d_ltab);
    }
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        hipGetLastError();
        hipFree(p->d_ltab);
        p->d_ltab = nullptr;
        return;
    }
    g.ltab = p->d_ltab;
    g.ltab_mode = p->phase_mode;
}

// Counts, pointers, speed, pitch, centre, frequencies and pulse of a geometry (host only).
static int check_geometry_basic(const spgm_geometry *gm, const char *who) {
    if (!gm) return fail(SPGM_E_INVALID, "%s: geometry is NULL", who);
    if (gm->n_tx < 1 || gm->n_rx < 1 || gm->n_freq < 1 || gm->nx < 1 || gm->ny < 1 || gm->nz < 1)
        return fail(SPGM_E_INVALID, "%s: every count must be >= 1", who);
    if (!gm->tx_xyz || !gm->rx_xyz || !gm->freq_hz)
        return fail(SPGM_E_INVALID, "%s: tx_xyz, rx_xyz and freq_hz must be non-NULL", who);
    if (!(std::isfinite(gm->c) && gm->c > 0)) return fail(SPGM_E_INVALID, "%s: c must be finite and > 0", who);
    if (!finite3(gm->centre) || !finite3(gm->pitch) || !(gm->pitch[0] > 0 && gm->pitch[1] > 0 && gm->pitch[2] > 0))
        return fail(SPGM_E_INVALID, "%s: centre must be finite and pitch > 0", who);
    for (int64_t f = 0; f < gm->n_freq; ++f) {
        if (!(std::isfinite(gm->freq_hz[f]) && gm->freq_hz[f] > 0))
            return fail(SPGM_E_INVALID, "%s: frequency %lld is not finite and > 0", who, (long long)f);
        if (gm->pulse && !(std::isfinite(gm->pulse[2 * f]) && std::isfinite(gm->pulse[2 * f + 1])))
            return fail(SPGM_E_INVALID, "%s: pulse %lld is not finite", who, (long long)f);
    }
    return SPGM_OK;
}

// Bound on the float32 argument of sin/cos in the compensated scheme, in turns: the reference
// phase reduced to [-1/2, 1/2] plus f/c times the two antennas' distance offsets, each at most the
// half-diagonal h of the voxel brick (triangle inequality).
static double phase_window_turns(const spgm_geometry *gm) {
    const double hx = 0.5 * (kBX - 1) * gm->pitch[0], hy = 0.5 * (kBY - 1) * gm->pitch[1];
    const double hz = 0.5 * (kBZ - 1) * gm->pitch[2];
    const double h = std::sqrt(hx * hx + hy * hy + hz * hz);
    double fmax = 0.0;
    for (int64_t f = 0; f < gm->n_freq; ++f) fmax = std::max(fmax, gm->freq_hz[f]);
    return 0.5 + 2.0 * (fmax / gm->c) * h;
}

int spgm_phase_window(const spgm_geometry *gm, double *turns) {
    int rc;
    if (!turns) return fail(SPGM_E_INVALID, "spgm_phase_window: turns is NULL");
    if ((rc = check_geometry_basic(gm, "spgm_phase_window"))) return rc;
    *turns = phase_window_turns(gm);
    return ok();
}

int spgm_plan_create(spgm_plan **out, const spgm_geometry *gm, int32_t phase_mode) {
    int rc;
    if (!out) return fail(SPGM_E_INVALID, "spgm_plan_create: out is NULL");
    *out = nullptr;
    if ((rc = check_geometry_basic(gm, "spgm_plan_create"))) return rc;
    if (phase_mode != SPGM_PHASE_COMP32 && phase_mode != SPGM_PHASE_F64 && phase_mode != SPGM_PHASE_NAIVE32)
        return fail(SPGM_E_INVALID, "spgm_plan_create: unknown phase mode %d", phase_mode);
    const int64_t T = gm->n_tx, R = gm->n_rx, F = gm->n_freq;
    const int64_t M = F * T * R;
    const int64_t N = (int64_t)gm->nx * gm->ny * gm->nz;
    if (M > INT32_MAX || N > INT32_MAX) return fail(SPGM_E_INVALID, "spgm_plan_create: M or N exceeds 2^31-1");
    if (std::min(T, R) > kMaxL || T + R > kMaxAnt)
        return fail(SPGM_E_UNSUPPORTED, "spgm_plan_create: needs min(T,R) <= %d and T+R <= %d", kMaxL, kMaxAnt);
    if (phase_mode == SPGM_PHASE_COMP32 && phase_window_turns(gm) > SPGM_COMP32_WINDOW_TURNS)
        return fail(SPGM_E_UNSUPPORTED,
                    "spgm_plan_create: the compensated float32 phase can reach %.2f turns for this pitch and "
                    "frequency, beyond the %.0f-turn window its accuracy holds in; use SPGM_PHASE_F64",
                    phase_window_turns(gm), (double)SPGM_COMP32_WINDOW_TURNS);
    // Antenna positions; voxels must stay away from every antenna (Eq. 2 divides by distances).
    const double lo[3] = {gm->centre[0] - 0.5 * (gm->nx - 1) * gm->pitch[0],
                          gm->centre[1] - 0.5 * (gm->ny - 1) * gm->pitch[1],
                          gm->centre[2] - 0.5 * (gm->nz - 1) * gm->pitch[2]};
    const double hi[3] = {lo[0] + (gm->nx - 1) * gm->pitch[0], lo[1] + (gm->ny - 1) * gm->pitch[1],
                          lo[2] + (gm->nz - 1) * gm->pitch[2]};
    const int dims[3] = {gm->nx, gm->ny, gm->nz};
    for (int64_t a = 0; a < T + R; ++a) {
        const double *ra = a < T ? gm->tx_xyz + 3 * a : gm->rx_xyz + 3 * (a - T);
        if (!finite3(ra)) return fail(SPGM_E_INVALID, "spgm_plan_create: antenna %lld is not finite", (long long)a);
        double box = 0.0;  // distance from the antenna to the grid's bounding box
        for (int k = 0; k < 3; ++k) {
            const double dd = std::max(0.0, std::max(lo[k] - ra[k], ra[k] - hi[k]));
            box += dd * dd;
        }
        if (std::sqrt(box) > 1e-9) continue;
        // Antenna inside the box: test the nearest grid voxel.
        double dmin2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            double i = std::nearbyint((ra[k] - lo[k]) / gm->pitch[k]);
            i = std::min<double>(std::max(i, 0.0), dims[k] - 1);
            const double dd = lo[k] + i * gm->pitch[k] - ra[k];
            dmin2 += dd * dd;
        }
        if (std::sqrt(dmin2) <= 1e-9)
            return fail(SPGM_E_INVALID, "spgm_plan_create: antenna %lld coincides with a voxel", (long long)a);
    }

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SPGM_E_DEVICE, "spgm_plan_create: no HIP device");
    spgm_plan *p = new spgm_plan();
    p->device = dev;
    p->scratch = scratch_address(dev);  // set-up of spgm_step_noalloc for this device
    p->phase_mode = phase_mode;
    p->M = M;
    p->N = N;
    Geo &g = p->geo;
    g.T = (int)T;
    g.R = (int)R;
    g.F = (int)F;
    g.nx = gm->nx;
    g.ny = gm->ny;
    g.nz = gm->nz;
    g.nbx = (gm->nx + kBX - 1) / kBX;
    g.nby = (gm->ny + kBY - 1) / kBY;
    g.nbz = (gm->nz + kBZ - 1) / kBZ;
    g.g_is_tx = R <= T ? 1 : 0;
    g.nG = g.g_is_tx ? (int)T : (int)R;
    g.nL = g.g_is_tx ? (int)R : (int)T;
    g.cx = gm->centre[0];
    g.cy = gm->centre[1];
    g.cz = gm->centre[2];
    g.px = gm->pitch[0];
    g.py = gm->pitch[1];
    g.pz = gm->pitch[2];
    const int64_t tiles = (int64_t)g.nbx * g.nby * g.nbz;
    p->n_tiles = (int)tiles;

    double *ant = new double[3 * (T + R)];
    std::memcpy(ant, gm->tx_xyz, sizeof(double) * 3 * T);
    std::memcpy(ant + 3 * T, gm->rx_xyz, sizeof(double) * 3 * R);
    double *kap = new double[F];
    float2 *q = new float2[F];
    const double inv4pi = 1.0 / (4.0 * 3.14159265358979323846);
    for (int64_t f = 0; f < F; ++f) {
        kap[f] = gm->freq_hz[f] / gm->c;
        const double pr = gm->pulse ? gm->pulse[2 * f] : 1.0;
        const double pi = gm->pulse ? gm->pulse[2 * f + 1] : 0.0;
        q[f] = make_float2((float)(pr * inv4pi), (float)(pi * inv4pi));
    }
    bool okk = hipMalloc(&p->d_ant, sizeof(double) * 3 * (T + R)) == hipSuccess &&
               hipMalloc(&p->d_kappa, sizeof(double) * F) == hipSuccess &&
               hipMalloc(&p->d_q, sizeof(float2) * F) == hipSuccess &&
               hipMalloc(&p->d_status, sizeof(int)) == hipSuccess;
    okk = okk && hipMemcpy(p->d_ant, ant, sizeof(double) * 3 * (T + R), hipMemcpyHostToDevice) == hipSuccess &&
          hipMemcpy(p->d_kappa, kap, sizeof(double) * F, hipMemcpyHostToDevice) == hipSuccess &&
          hipMemcpy(p->d_q, q, sizeof(float2) * F, hipMemcpyHostToDevice) == hipSuccess &&
          hipMemset(p->d_status, 0, sizeof(int)) == hipSuccess;
    delete[] ant;
    delete[] kap;
    delete[] q;
    if (!okk) {
        spgm_plan_destroy(p);
        return fail(SPGM_E_NOMEM, "spgm_plan_create: device allocation or copy failed");
    }
    g.ant = p->d_ant;
    g.kappa = p->d_kappa;
    g.q = p->d_q;
    const size_t A = (size_t)(T + R);
    p->lds_bytes = tile_lds(g, kWaves);
    if (p->lds_bytes > (size_t)kMaxLds) {
        spgm_plan_destroy(p);
        return fail(SPGM_E_UNSUPPORTED, "spgm_plan_create: LDS footprint exceeds 160 KiB");
    }
    // Two work-groups of eight waves per compute unit (four waves per SIMD) where their brick
    // tables fit twice in LDS; otherwise one work-group of sixteen waves keeps four per SIMD.
    p->tile_waves = (2 * p->lds_bytes > (size_t)kMaxLds && tile_lds(g, 16) <= (size_t)kMaxLds) ? 16 : 8;
    hipFuncSetAttribute((const void *)k_sort_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)(sizeof(unsigned long long) * kSortChunk));
    const void *tile_kernels8[] = {
        (const void *)k_fwd_tile<SPGM_PHASE_COMP32, 8>, (const void *)k_fwd_tile<SPGM_PHASE_F64, 8>,
        (const void *)k_fwd_tile<SPGM_PHASE_NAIVE32, 8>, (const void *)k_adj_tile<SPGM_PHASE_COMP32, 8>,
        (const void *)k_adj_tile<SPGM_PHASE_F64, 8>, (const void *)k_adj_tile<SPGM_PHASE_NAIVE32, 8>};
    for (const void *k : tile_kernels8)
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p->lds_bytes);
    const void *tile_kernels16[] = {
        (const void *)k_fwd_tile<SPGM_PHASE_COMP32, 16>, (const void *)k_fwd_tile<SPGM_PHASE_F64, 16>,
        (const void *)k_fwd_tile<SPGM_PHASE_NAIVE32, 16>, (const void *)k_adj_tile<SPGM_PHASE_COMP32, 16>,
        (const void *)k_adj_tile<SPGM_PHASE_F64, 16>, (const void *)k_adj_tile<SPGM_PHASE_NAIVE32, 16>};
    for (const void *k : tile_kernels16)
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    const void *mm_kernels[] = {
        (const void *)k_mm_fwd<SPGM_MM_BF16, 1>, (const void *)k_mm_fwd<SPGM_MM_BF16, 2>,
        (const void *)k_mm_fwd<SPGM_MM_BF16, 3>, (const void *)k_mm_fwd<SPGM_MM_BF16, 4>,
        (const void *)k_mm_fwd<SPGM_MM_FP16, 1>, (const void *)k_mm_fwd<SPGM_MM_FP16, 2>,
        (const void *)k_mm_fwd<SPGM_MM_FP16, 3>, (const void *)k_mm_fwd<SPGM_MM_FP16, 4>,
        (const void *)k_mm_adj<SPGM_MM_BF16>, (const void *)k_mm_adj<SPGM_MM_FP16>};
    for (const void *k : mm_kernels) hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    const void *mm_rows_kernels[] = {
        (const void *)k_mm_fwd_rows<SPGM_MM_BF16, 1>, (const void *)k_mm_fwd_rows<SPGM_MM_BF16, 2>,
        (const void *)k_mm_fwd_rows<SPGM_MM_BF16, 3>, (const void *)k_mm_fwd_rows<SPGM_MM_BF16, 4>,
        (const void *)k_mm_fwd_rows<SPGM_MM_FP16, 1>, (const void *)k_mm_fwd_rows<SPGM_MM_FP16, 2>,
        (const void *)k_mm_fwd_rows<SPGM_MM_FP16, 3>, (const void *)k_mm_fwd_rows<SPGM_MM_FP16, 4>};
    for (const void *k : mm_rows_kernels) hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    const void *sf_kernels[] = {(const void *)k_sf_fwd<kSFItemsSmall>, (const void *)k_sf_fwd<kSFItems>,
                                (const void *)k_sf_adj<kSFItemsSmall, 1>, (const void *)k_sf_adj<kSFItems, 2>};
    for (const void *k : sf_kernels)
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sf_lds_bytes((int)A));
    hipGetLastError();
    build_ltab(p);
    *out = p;
    return ok();
}

int spgm_plan_opts_init(spgm_plan_opts *o) {
    if (!o) return fail(SPGM_E_INVALID, "spgm_plan_opts_init: opts is NULL");
    o->phase_mode = SPGM_PHASE_COMP32;
    o->device = -1;
    o->tune_cache = nullptr;
    return ok();
}

int spgm_plan_create_ex(spgm_plan **out, const spgm_geometry *gm, const spgm_plan_opts *o) {
    if (!o) return fail(SPGM_E_INVALID, "spgm_plan_create_ex: opts is NULL");
    int rc;
    if (o->device >= 0) {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || o->device >= n)
            return fail(SPGM_E_INVALID, "spgm_plan_create_ex: device %d is not present", o->device);
        DeviceGuard guard(o->device);
        rc = spgm_plan_create(out, gm, o->phase_mode);
    } else {
        rc = spgm_plan_create(out, gm, o->phase_mode);
    }
    if (rc == SPGM_OK && o->tune_cache) (*out)->tune_cache = o->tune_cache;
    return rc;
}

int spgm_plan_destroy(spgm_plan *p) {
    if (!p) return ok();
    DeviceGuard guard(p->device);
    hipDeviceSynchronize();
    hipFree(p->d_ant);
    hipFree(p->d_kappa);
    hipFree(p->d_q);
    hipFree(p->d_status);
    hipFree(p->d_ltab);
    hipFree(p->d_srt);
    hipFree(p->d_part);
    hipFree(p->d_rs);
    hipFree(p->d_gpart);
    hipFree(p->d_s_alt);
    hipFree(p->d_srt_all);
    hipFree(p->d_vjp);
    hipFree(p->d_tv_b);
    hipFree(p->d_tv_state);
    hipFree(p->d_vjp_part);
    hipFree(p->d_mm_s);
    hipFree(p->d_gtab);
    hipFree(p->d_mm_part);
    hipFree(p->d_mm_r);
    hipFree(p->d_mm_gpart);
    hipFree(p->d_sf_rows);
    hipFree(p->d_tol_snap);
    hipFree(p->d_tol_part);
    hipFree(p->d_tol_rec);
    hipFree(p->d_tol_rows);
    drop_graph(p);
    if (p->cap_stream) hipStreamDestroy(p->cap_stream);
    for (hipEvent_t e : p->ev_fwd) hipEventDestroy(e);
    for (hipEvent_t e : p->ev_adj) hipEventDestroy(e);
    delete p;
    return ok();
}

int spgm_plan_dims(const spgm_plan *p, int64_t *M, int64_t *N) {
    if (!p) return fail(SPGM_E_INVALID, "spgm_plan_dims: plan is NULL");
    if (M) *M = p->M;
    if (N) *N = p->N;
    return ok();
}

int spgm_forward(spgm_plan *p, const int32_t *rows, int32_t B, const void *s, void *y, void *stream) {
    int rc;
    if ((rc = check_common(p, rows, B))) return rc;
    if (!s || !y) return fail(SPGM_E_INVALID, "spgm_forward: s and y must be non-NULL");
    DeviceGuard guard(p->device);
    if ((rc = ensure_workspace(p, B))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = run_sort(p, rows, B, 1, p->d_srt, st))) return rc;
    if ((rc = run_forward_partials(p, p->d_srt, (const float2 *)s, B, st))) return rc;
    if ((rc = run_row_reduce(p, p->d_srt, rows, B, nullptr, (float2 *)y, nullptr, st))) return rc;
    return ok();
}

int spgm_adjoint(spgm_plan *p, const int32_t *rows, int32_t B, const void *r, void *g, void *stream) {
    int rc;
    if ((rc = check_common(p, rows, B))) return rc;
    if (!r || !g) return fail(SPGM_E_INVALID, "spgm_adjoint: r and g must be non-NULL");
    DeviceGuard guard(p->device);
    if ((rc = ensure_workspace(p, B))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = run_sort(p, rows, B, 1, p->d_srt, st))) return rc;
    k_gather_scale<<<(B + 255) / 256, 256, 0, st>>>(p->geo, p->d_srt, B, (const float2 *)r, p->d_rs);
    if ((rc = launch_check("gather"))) return rc;
    if ((rc = run_adjoint_partials(p, p->d_srt, B, st))) return rc;
    k_col_reduce<<<(int)((p->N + 255) / 256), 256, 0, st>>>(p->d_gpart, adj_splits(p, B), (int)p->N, (float2 *)g,
                                                             nullptr, 0.f, 0.f);
    if ((rc = launch_check("column reduce"))) return rc;
    return ok();
}

static int check_step_args(const void *y, const void *s, float eta, float alpha) {
    if (!y || !s) return fail(SPGM_E_INVALID, "spgm: y and s must be non-NULL");
    if (!(std::isfinite(eta) && eta > 0)) return fail(SPGM_E_INVALID, "spgm: eta must be finite and > 0");
    if (!(std::isfinite(alpha) && alpha >= 0)) return fail(SPGM_E_INVALID, "spgm: alpha must be finite and >= 0");
    return SPGM_OK;
}

int spgm_step(spgm_plan *p, const int32_t *rows, int32_t B, const void *y, void *s, float eta, float alpha,
              void *stream) {
    int rc;
    if ((rc = check_common(p, rows, B))) return rc;
    if ((rc = check_step_args(y, s, eta, alpha))) return rc;
    DeviceGuard guard(p->device);
    if ((rc = ensure_workspace(p, B))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = run_sort(p, rows, B, 1, p->d_srt, st))) return rc;
    if ((rc = step_sorted(p, p->d_srt, rows, B, (const float2 *)y, (float2 *)s, eta, alpha, st, plan_work(p))))
        return rc;
    return ok();
}

int spgm_step_grad(spgm_plan *p, const int32_t *rows, int32_t B, const void *y, void *s, float eta, float alpha,
                   void *g, void *stream) {
    int rc;
    if ((rc = check_common(p, rows, B))) return rc;
    if ((rc = check_step_args(y, s, eta, alpha))) return rc;
    if (!g) return fail(SPGM_E_INVALID, "spgm_step_grad: g must be non-NULL");
    DeviceGuard guard(p->device);
    if ((rc = ensure_workspace(p, B))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = run_sort(p, rows, B, 1, p->d_srt, st))) return rc;
    if ((rc = run_forward_partials(p, p->d_srt, (const float2 *)s, B, st))) return rc;
    if ((rc = run_row_reduce(p, p->d_srt, rows, B, (const float2 *)y, nullptr, p->d_rs, st))) return rc;
    if ((rc = run_adjoint_partials(p, p->d_srt, B, st))) return rc;
    k_col_reduce<<<(int)((p->N + 255) / 256), 256, 0, st>>>(p->d_gpart, adj_splits(p, B), (int)p->N, (float2 *)g,
                                                             (float2 *)s, eta / (float)B, alpha);
    if ((rc = launch_check("column reduce"))) return rc;
    return ok();
}

int spgm_step_noalloc(spgm_plan *p, const int32_t *rows, int32_t B, const void *y, void *s, float eta, float alpha,
                      void *stream) {
    int rc;
    if ((rc = check_common(p, rows, B))) return rc;
    if ((rc = check_step_args(y, s, eta, alpha))) return rc;
    if (!p->scratch)
        return fail(SPGM_E_DEVICE, "spgm_step_noalloc: the scratch array has no device address on device %d",
                    p->device);
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t b_srt = al(sizeof(int4) * (size_t)B);
    const size_t b_part = al(sizeof(float2) * (size_t)p->n_tiles * B);
    const size_t b_rs = al(sizeof(float2) * (size_t)B);
    const size_t b_gpart = al(sizeof(float2) * (size_t)adj_splits(p, B) * p->N);
    const size_t need = b_srt + b_part + b_rs + b_gpart;
    if (need > kScratchBytes)
        return fail(SPGM_E_UNSUPPORTED,
                    "spgm_step_noalloc: B=%d on %d voxel bricks needs %zu bytes of workspace, more than the %zu-byte "
                    "scratch array (use spgm_step)", B, p->n_tiles, need, kScratchBytes);
    DeviceGuard guard(p->device);
    char *base = p->scratch;
    int4 *srt = reinterpret_cast<int4 *>(base);
    const StepWork w{reinterpret_cast<float2 *>(base + b_srt), reinterpret_cast<float2 *>(base + b_srt + b_part),
                     reinterpret_cast<float2 *>(base + b_srt + b_part + b_rs)};
    // Every word of the workspace that a kernel reads is written earlier in this call, so the
    // previous call's contents need no clearing.  Timing events are not created here.
    const bool timing = p->timing;
    p->timing = false;
    hipStream_t st = (hipStream_t)stream;
    rc = run_sort(p, rows, B, 1, srt, st);
    if (!rc) rc = step_sorted(p, srt, rows, B, (const float2 *)y, (float2 *)s, eta, alpha, st, w);
    p->timing = timing;
    if (rc) return rc;
    return ok();
}

// Issue the launches of an iters-iteration solve on `st` (workspace already sized).  The
// proximal step of iteration k is applied by the forward of iteration k + 1 to the voxels it
// reads (one launch fewer per iteration, same arithmetic as the column reduction); iterates
// alternate between s and the plan's second buffer, and the last step is a column reduction
// into s.  Results are bitwise those of iters calls of the single step.
static int solve_launches(spgm_plan *p, const int32_t *rows, int iters, int B, const float2 *y, float2 *s, float eta,
                          float alpha, hipStream_t st) {
    int rc;
    float2 *const buf[2] = {s, p->d_s_alt};
    const float step = eta / (float)B;
    const int nsplit = adj_splits(p, B);
    // The minibatch table is an input, so all of its minibatches are sorted ahead in one launch
    // per batch of iterations; the iterations then run back to back on the sorted tables.
    const int per = (int)std::max<size_t>(1, std::min<size_t>((size_t)iters, kSolveSortRows / (size_t)B));
    for (int k0 = 0; k0 < iters; k0 += per) {
        const int cnt = std::min(per, iters - k0);
        const int32_t *rk = rows + (size_t)k0 * B;
        if ((rc = run_sort(p, rk, B, cnt, p->d_srt_all, st))) return rc;
        for (int k = 0; k < cnt; ++k) {
            const int it = k0 + k;
            const int4 *srt = p->d_srt_all + (size_t)k * B;
            const SStep up = it == 0 ? SStep{} : SStep{p->d_gpart, buf[it & 1], nsplit, (int)p->N, step, alpha};
            const float2 *s_prev = it == 0 ? s : buf[(it - 1) & 1];
            if ((rc = run_forward_partials(p, srt, s_prev, B, st, up))) return rc;
            if ((rc = run_row_reduce(p, srt, rk + (size_t)k * B, B, y, nullptr, p->d_rs, st))) return rc;
            if ((rc = run_adjoint_partials(p, srt, B, st))) return rc;
        }
    }
    k_col_reduce_to<<<(int)((p->N + 255) / 256), 256, 0, st>>>(p->d_gpart, nsplit, (int)p->N, buf[(iters - 1) & 1], s,
                                                                step, alpha);
    return launch_check("column reduce");
}

static int solve_prepare(spgm_plan *p, const int32_t *rows, int32_t iters, int32_t B, const void *y, void *s,
                         float eta, float alpha) {
    int rc;
    if ((rc = check_common(p, rows, B))) return rc;
    if ((rc = check_step_args(y, s, eta, alpha))) return rc;
    if (iters < 0) return fail(SPGM_E_INVALID, "spgm_solve: iters must be >= 0");
    if ((rc = ensure_workspace(p, B))) return rc;
    if (iters == 0) return SPGM_OK;
    if (!p->d_s_alt && hipMalloc(&p->d_s_alt, sizeof(float2) * (size_t)p->N) != hipSuccess) {
        p->d_s_alt = nullptr;
        return fail(SPGM_E_NOMEM, "spgm_solve: iterate buffer allocation failed");
    }
    const size_t per = std::max<size_t>(1, std::min<size_t>((size_t)iters, kSolveSortRows / (size_t)B));
    return ensure_sorted_batch(p, per * B);
}

int spgm_solve(spgm_plan *p, const int32_t *rows, int32_t iters, int32_t B, const void *y, void *s, float eta,
               float alpha, void *stream) {
    int rc;
    if (!p) return fail(SPGM_E_INVALID, "spgm: plan is NULL");
    DeviceGuard guard(p->device);
    if ((rc = solve_prepare(p, rows, iters, B, y, s, eta, alpha))) return rc;
    if (iters == 0) return ok();
    if ((rc = solve_launches(p, rows, iters, B, (const float2 *)y, (float2 *)s, eta, alpha, (hipStream_t)stream)))
        return rc;
    return ok();
}

int spgm_prox(spgm_plan *p, const spgm_regularizer *reg, void *v, float alpha, void *stream) {
    int rc;
    if (!p) return fail(SPGM_E_INVALID, "spgm: plan is NULL");
    if ((rc = check_reg(reg))) return rc;
    if (!v) return fail(SPGM_E_INVALID, "spgm_prox: v must be non-NULL");
    if (!(std::isfinite(alpha) && alpha >= 0)) return fail(SPGM_E_INVALID, "spgm: alpha must be finite and >= 0");
    DeviceGuard guard(p->device);
    hipStream_t st = (hipStream_t)stream;
    if (reg->kind == SPGM_REG_TV_MAGNITUDE) {
        if ((rc = ensure_tv(p))) return rc;
        if ((rc = run_tv_prox(p, (float2 *)v, alpha, reg->tv_iters, st))) return rc;
        return ok();
    }
    const float scale = reg->kind == SPGM_REG_ELASTIC_NET ? elastic_scale(alpha, reg->mu) : 1.f;
    k_prox_elastic<<<(int)((p->N + kRegThreads - 1) / kRegThreads), kRegThreads, 0, st>>>((float2 *)v, (int)p->N,
                                                                                        alpha, scale);
    if ((rc = launch_check("prox"))) return rc;
    return ok();
}

int spgm_step_reg(spgm_plan *p, const spgm_regularizer *reg, const int32_t *rows, int32_t B, const void *y, void *s,
                  float eta, float alpha, void *stream) {
    int rc;
    if ((rc = check_common(p, rows, B))) return rc;
    if ((rc = check_step_args(y, s, eta, alpha))) return rc;
    if ((rc = check_reg(reg))) return rc;
    DeviceGuard guard(p->device);
    if ((rc = ensure_workspace(p, B))) return rc;
    if (reg->kind == SPGM_REG_TV_MAGNITUDE && (rc = ensure_tv(p))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = run_sort(p, rows, B, 1, p->d_srt, st))) return rc;
    if ((rc = step_sorted_reg(p, p->d_srt, rows, B, (const float2 *)y, (float2 *)s, eta, alpha, *reg, st)))
        return rc;
    return ok();
}

int spgm_solve_reg(spgm_plan *p, const spgm_regularizer *reg, const int32_t *rows, int32_t iters, int32_t B,
                   const void *y, void *s, float eta, float alpha, void *stream) {
    int rc;
    if (!p) return fail(SPGM_E_INVALID, "spgm: plan is NULL");
    if ((rc = check_reg(reg))) return rc;
    DeviceGuard guard(p->device);
    if ((rc = solve_prepare(p, rows, iters, B, y, s, eta, alpha))) return rc;
    if (iters == 0) return ok();
    if (reg->kind == SPGM_REG_TV_MAGNITUDE && (rc = ensure_tv(p))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int per = (int)std::max<size_t>(1, std::min<size_t>((size_t)iters, kSolveSortRows / (size_t)B));
    for (int k0 = 0; k0 < iters; k0 += per) {
        const int cnt = std::min(per, iters - k0);
        const int32_t *rk = rows + (size_t)k0 * B;
        if ((rc = run_sort(p, rk, B, cnt, p->d_srt_all, st))) return rc;
        for (int k = 0; k < cnt; ++k) {
            if ((rc = step_sorted_reg(p, p->d_srt_all + (size_t)k * B, rk + (size_t)k * B, B, (const float2 *)y,
                                      (float2 *)s, eta, alpha, *reg, st)))
                return rc;
        }
    }
    return ok();
}

int spgm_solve_graph(spgm_plan *p, const int32_t *rows, int32_t iters, int32_t B, const void *y, void *s, float eta,
                     float alpha, void *stream) {
    int rc;
    if (!p) return fail(SPGM_E_INVALID, "spgm: plan is NULL");
    DeviceGuard guard(p->device);
    if ((rc = solve_prepare(p, rows, iters, B, y, s, eta, alpha))) return rc;
    if (iters == 0) return ok();
    const bool same = p->graph_exec && p->graph_key.rows == rows && p->graph_key.iters == iters &&
                      p->graph_key.B == B && p->graph_key.y == y && p->graph_key.s == s &&
                      p->graph_key.eta == eta && p->graph_key.alpha == alpha;
    if (!same) {
        drop_graph(p);
        if (!p->cap_stream && hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
            return fail(SPGM_E_DEVICE, "spgm_solve_graph: stream creation failed");
        const bool timing = p->timing;
        p->timing = false;  // no event records inside the captured graph
        if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            p->timing = timing;
            return fail(SPGM_E_DEVICE, "spgm_solve_graph: capture failed to start");
        }
        rc = solve_launches(p, rows, iters, B, (const float2 *)y, (float2 *)s, eta, alpha, p->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
        p->timing = timing;
        if (rc) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess || !g) return fail(SPGM_E_DEVICE, "spgm_solve_graph: capture failed: %s", hipGetErrorString(e));
        p->graph = g;
        if (hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(g);
            p->graph = nullptr;
            return fail(SPGM_E_DEVICE, "spgm_solve_graph: graph instantiation failed");
        }
        p->graph_key.rows = rows;
        p->graph_key.iters = iters;
        p->graph_key.B = B;
        p->graph_key.y = y;
        p->graph_key.s = s;
        p->graph_key.eta = eta;
        p->graph_key.alpha = alpha;
    }
    const hipError_t e = hipGraphLaunch(p->graph_exec, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SPGM_E_DEVICE, "spgm_solve_graph: launch failed: %s", hipGetErrorString(e));
    return ok();
}

// ---------------------------------------------------------------- solve to the termination rule
// One group of `cnt` iterations on rows[0 .. cnt*B): sort, then per iteration the forward, the
// residual, the adjoint and the column reduction that also forms the iteration's change record
// rec[2j] = sum (|s^k| - |s^{k-1}|)^2, rec[2j+1] = sum |s^{k-1}|^2 (fixed-order float64 sums).
static int tol_group_launches(spgm_plan *p, const int32_t *rows, int cnt, int B, const float2 *y, float2 *s,
                              float eta, float alpha, double *rec, hipStream_t st) {
    int rc;
    if ((rc = run_sort(p, rows, B, cnt, p->d_srt_all, st))) return rc;
    const int nb = (int)((p->N + kChgThreads - 1) / kChgThreads);
    for (int j = 0; j < cnt; ++j) {
        const int4 *srt = p->d_srt_all + (size_t)j * B;
        if ((rc = run_forward_partials(p, srt, s, B, st))) return rc;
        if ((rc = run_row_reduce(p, srt, rows + (size_t)j * B, B, y, nullptr, p->d_rs, st))) return rc;
        if ((rc = run_adjoint_partials(p, srt, B, st))) return rc;
        k_col_reduce_change<<<nb, kChgThreads, 0, st>>>(p->d_gpart, adj_splits(p, B), (int)p->N, s, eta / (float)B,
                                                        alpha, p->d_tol_part);
        if ((rc = launch_check("column reduce (change)"))) return rc;
        k_sum_partials<<<1, 256, 0, st>>>(p->d_tol_part, nb, rec + 2 * j, rec + 2 * j + 1);
        if ((rc = launch_check("change sum"))) return rc;
    }
    return SPGM_OK;
}

static int tol_prepare(spgm_plan *p, int group, int B) {
    int rc;
    const size_t nb = (size_t)((p->N + kChgThreads - 1) / kChgThreads);
    if (!p->d_tol_snap) {
        if (hipMalloc(&p->d_tol_snap, sizeof(float2) * (size_t)p->N) != hipSuccess ||
            hipMalloc(&p->d_tol_part, sizeof(double) * 2 * nb) != hipSuccess) {
            hipFree(p->d_tol_snap);
            p->d_tol_snap = nullptr;
            p->d_tol_part = nullptr;
            return fail(SPGM_E_NOMEM, "spgm_solve_tol: workspace allocation failed");
        }
    }
    if ((size_t)group > p->tol_group_cap) {
        drop_graph(p);
        hipFree(p->d_tol_rec);
        p->d_tol_rec = nullptr;
        p->tol_group_cap = 0;
        if (hipMalloc(&p->d_tol_rec, sizeof(double) * 2 * ((size_t)group + 1)) != hipSuccess)
            return fail(SPGM_E_NOMEM, "spgm_solve_tol: record allocation failed");
        p->tol_group_cap = (size_t)group;
    }
    if ((size_t)group * B > p->tol_rows_cap) {
        drop_graph(p);
        hipFree(p->d_tol_rows);
        p->d_tol_rows = nullptr;
        p->tol_rows_cap = 0;
        if (hipMalloc(&p->d_tol_rows, sizeof(int32_t) * (size_t)group * B) != hipSuccess)
            return fail(SPGM_E_NOMEM, "spgm_solve_tol: row buffer allocation failed");
        p->tol_rows_cap = (size_t)group * B;
    }
    if ((rc = ensure_sorted_batch(p, (size_t)group * B))) return rc;
    return SPGM_OK;
}

// Graph of one full group on the plan's row buffer (captured once per group size, B, y, s, eta,
// alpha; replayed after the group's rows are copied into the buffer).
static int tol_group_graph(spgm_plan *p, int group, int B, const float2 *y, float2 *s, float eta, float alpha,
                           hipStream_t st) {
    const bool same = p->tol_exec && p->tol_key.group == group && p->tol_key.B == B && p->tol_key.y == y &&
                      p->tol_key.s == s && p->tol_key.eta == eta && p->tol_key.alpha == alpha;
    if (!same) {
        if (p->tol_exec) hipGraphExecDestroy(p->tol_exec);
        if (p->tol_graph) hipGraphDestroy(p->tol_graph);
        p->tol_exec = nullptr;
        p->tol_graph = nullptr;
        if (!p->cap_stream && hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
            return fail(SPGM_E_DEVICE, "spgm_solve_tol: stream creation failed");
        const bool timing = p->timing;
        p->timing = false;
        if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            p->timing = timing;
            return fail(SPGM_E_DEVICE, "spgm_solve_tol: capture failed to start");
        }
        int rc = tol_group_launches(p, p->d_tol_rows, group, B, y, s, eta, alpha, p->d_tol_rec, p->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
        p->timing = timing;
        if (rc) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess || !g) return fail(SPGM_E_DEVICE, "spgm_solve_tol: capture failed: %s", hipGetErrorString(e));
        if (hipGraphInstantiate(&p->tol_exec, g, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(g);
            return fail(SPGM_E_DEVICE, "spgm_solve_tol: graph instantiation failed");
        }
        p->tol_graph = g;
        p->tol_key.group = group;
        p->tol_key.B = B;
        p->tol_key.y = y;
        p->tol_key.s = s;
        p->tol_key.eta = eta;
        p->tol_key.alpha = alpha;
    }
    const hipError_t e = hipGraphLaunch(p->tol_exec, st);
    if (e != hipSuccess) return fail(SPGM_E_DEVICE, "spgm_solve_tol: graph launch failed: %s", hipGetErrorString(e));
    return SPGM_OK;
}

int spgm_solve_tol(spgm_plan *p, const int32_t *rows, int32_t iters, int32_t B, const void *y, void *s, float eta,
                   float alpha, double tol, int32_t check_every, int32_t use_graph, int32_t *iters_done,
                   double *changes, void *stream) {
    int rc;
    if ((rc = check_common(p, rows, B))) return rc;
    if ((rc = check_step_args(y, s, eta, alpha))) return rc;
    if (!iters_done) return fail(SPGM_E_INVALID, "spgm_solve_tol: iters_done is NULL");
    if (iters < 0) return fail(SPGM_E_INVALID, "spgm_solve_tol: iters must be >= 0");
    if (check_every < 1) return fail(SPGM_E_INVALID, "spgm_solve_tol: check_every must be >= 1");
    if (std::isnan(tol)) return fail(SPGM_E_INVALID, "spgm_solve_tol: tol is NaN");
    *iters_done = 0;
    DeviceGuard guard(p->device);
    if ((rc = ensure_workspace(p, B))) return rc;
    if (iters == 0) return ok();
    const int group = std::max(1, std::min<int>(std::min(check_every, iters), (int)(kSolveSortRows / (size_t)B)));
    if ((rc = tol_prepare(p, group, B))) return rc;
    hipStream_t st = (hipStream_t)stream;
    float2 *sv = (float2 *)s;
    const float2 *yv = (const float2 *)y;
    const size_t sbytes = sizeof(float2) * (size_t)p->N;
    std::vector<double> rec(2 * (size_t)group);
    const double tol2 = tol > 0 ? tol * tol : -1.0;
    for (int k = 0; k < iters;) {
        const int cnt = std::min(group, iters - k);
        const int32_t *rk = rows + (size_t)k * B;
        if (hipMemcpyAsync(p->d_tol_snap, sv, sbytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return fail(SPGM_E_DEVICE, "spgm_solve_tol: iterate copy failed");
        const int32_t *rows_used = rk;
        if (use_graph && cnt == group) {
            if (hipMemcpyAsync(p->d_tol_rows, rk, sizeof(int32_t) * (size_t)cnt * B, hipMemcpyDeviceToDevice, st) !=
                hipSuccess)
                return fail(SPGM_E_DEVICE, "spgm_solve_tol: row copy failed");
            if ((rc = tol_group_graph(p, group, B, yv, sv, eta, alpha, st))) return rc;
            rows_used = p->d_tol_rows;
        } else if ((rc = tol_group_launches(p, rk, cnt, B, yv, sv, eta, alpha, p->d_tol_rec, st))) {
            return rc;
        }
        if (hipMemcpyAsync(rec.data(), p->d_tol_rec, sizeof(double) * 2 * cnt, hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return fail(SPGM_E_DEVICE, "spgm_solve_tol: record read failed");
        int stop = -1;
        bool bad = false;
        for (int j = 0; j < cnt; ++j) {
            const double d2 = rec[2 * j], o2 = rec[2 * j + 1];
            if (changes) changes[k + j] = o2 > 0 ? std::sqrt(d2 / o2) : HUGE_VAL;
            if (!std::isfinite(d2) || !std::isfinite(o2)) {
                stop = j;
                bad = true;
                break;
            }
            if (d2 < tol2 * o2) {
                stop = j;
                break;
            }
        }
        if (stop < 0) {
            k += cnt;
            continue;
        }
        if (stop < cnt - 1) {
            // Back to the group's first iterate and forward to the stopping one: the same kernels
            // on the same sorted rows, so the iterate is bitwise the one the rule was met at.
            if (hipMemcpyAsync(sv, p->d_tol_snap, sbytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
                return fail(SPGM_E_DEVICE, "spgm_solve_tol: iterate restore failed");
            const int nb = (int)((p->N + kChgThreads - 1) / kChgThreads);
            for (int j = 0; j <= stop; ++j) {
                const int4 *srt = p->d_srt_all + (size_t)j * B;
                if ((rc = run_forward_partials(p, srt, sv, B, st))) return rc;
                if ((rc = run_row_reduce(p, srt, rows_used + (size_t)j * B, B, yv, nullptr, p->d_rs, st))) return rc;
                if ((rc = run_adjoint_partials(p, srt, B, st))) return rc;
                k_col_reduce_change<<<nb, kChgThreads, 0, st>>>(p->d_gpart, adj_splits(p, B), (int)p->N, sv,
                                                                eta / (float)B, alpha, p->d_tol_part);
                if ((rc = launch_check("column reduce (change)"))) return rc;
            }
            if (hipStreamSynchronize(st) != hipSuccess) return fail(SPGM_E_DEVICE, "spgm_solve_tol: replay failed");
        }
        *iters_done = k + stop + 1;
        if (bad)
            return fail(SPGM_E_NONFINITE, "spgm_solve_tol: the iterate of iteration %d is not finite", k + stop + 1);
        return ok();
    }
    *iters_done = iters;
    return ok();
}

// Backward of one unrolled iteration from the gradient g = A_B^H (A_B s - y_B) at its entering
// iterate (rows already sorted into p->d_srt): prox VJP, h = A_B^H A_B zbar, sbar = zbar - step h,
// and the fixed-order sums of the parameter gradients.
static int vjp_from_gradient(spgm_plan *p, const int32_t *rows, int B, const float2 *s, const float2 *g, float eta,
                             float tau, const float2 *sbar_next, float2 *sbar, double *eta_bar, double *tau_bar,
                             hipStream_t st) {
    int rc;
    const int N = (int)p->N;
    float2 *zbar = p->d_vjp + N, *h = p->d_vjp + 2 * (size_t)N;
    const int nb = (N + kVjpThreads - 1) / kVjpThreads;
    const float step = eta / (float)B;
    k_prox_vjp<<<nb, kVjpThreads, 0, st>>>(s, g, sbar_next, N, step, tau, 1.0f / (float)B, zbar, p->d_vjp_part);
    if ((rc = launch_check("prox vjp"))) return rc;
    if ((rc = run_forward_partials(p, p->d_srt, zbar, B, st))) return rc;
    if ((rc = run_row_reduce(p, p->d_srt, rows, B, nullptr, nullptr, p->d_rs, st))) return rc;
    if ((rc = run_adjoint_partials(p, p->d_srt, B, st))) return rc;
    k_col_reduce<<<(N + 255) / 256, 256, 0, st>>>(p->d_gpart, adj_splits(p, B), N, h, nullptr, 0.f, 0.f);
    if ((rc = launch_check("column reduce"))) return rc;
    k_axpy_out<<<(N + 255) / 256, 256, 0, st>>>(zbar, h, N, step, sbar);
    if ((rc = launch_check("axpy"))) return rc;
    k_sum_partials<<<1, 256, 0, st>>>(p->d_vjp_part, nb, eta_bar, tau_bar);
    return launch_check("sum partials");
}

static int vjp_check(spgm_plan *p, const int32_t *rows, int B, const void *s, const void *other, float eta, float tau,
                     const void *sbar_next, const void *sbar, const double *eta_bar, const double *tau_bar,
                     const char *who) {
    int rc;
    if ((rc = check_common(p, rows, B))) return rc;
    if (!other || !s || !sbar_next || !sbar || !eta_bar || !tau_bar)
        return fail(SPGM_E_INVALID, "%s: NULL pointer argument", who);
    if (!(std::isfinite(eta) && eta > 0) || !(std::isfinite(tau) && tau >= 0))
        return fail(SPGM_E_INVALID, "%s: eta must be > 0 and tau >= 0, finite", who);
    return SPGM_OK;
}

int spgm_unrolled_vjp_step(spgm_plan *p, const int32_t *rows, int32_t B, const void *y, const void *s,
                           float eta, float tau, const void *sbar_next, void *sbar, double *eta_bar,
                           double *tau_bar, void *stream) {
    int rc;
    if ((rc = vjp_check(p, rows, B, s, y, eta, tau, sbar_next, sbar, eta_bar, tau_bar, "spgm_unrolled_vjp_step")))
        return rc;
    DeviceGuard guard(p->device);
    if ((rc = ensure_workspace(p, B)) || (rc = ensure_vjp(p))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int N = (int)p->N;
    float2 *g = p->d_vjp;
    // recompute g = A_B^H (A_B s - y_B) at the iterate entering the iteration
    if ((rc = run_sort(p, rows, B, 1, p->d_srt, st))) return rc;
    if ((rc = run_forward_partials(p, p->d_srt, (const float2 *)s, B, st))) return rc;
    if ((rc = run_row_reduce(p, p->d_srt, rows, B, (const float2 *)y, nullptr, p->d_rs, st))) return rc;
    if ((rc = run_adjoint_partials(p, p->d_srt, B, st))) return rc;
    k_col_reduce<<<(N + 255) / 256, 256, 0, st>>>(p->d_gpart, adj_splits(p, B), N, g, nullptr, 0.f, 0.f);
    if ((rc = launch_check("column reduce"))) return rc;
    if ((rc = vjp_from_gradient(p, rows, B, (const float2 *)s, g, eta, tau, (const float2 *)sbar_next, (float2 *)sbar,
                                eta_bar, tau_bar, st)))
        return rc;
    return ok();
}

int spgm_unrolled_vjp_step_g(spgm_plan *p, const int32_t *rows, int32_t B, const void *s, const void *g, float eta,
                             float tau, const void *sbar_next, void *sbar, double *eta_bar, double *tau_bar,
                             void *stream) {
    int rc;
    if ((rc = vjp_check(p, rows, B, s, g, eta, tau, sbar_next, sbar, eta_bar, tau_bar, "spgm_unrolled_vjp_step_g")))
        return rc;
    DeviceGuard guard(p->device);
    if ((rc = ensure_workspace(p, B)) || (rc = ensure_vjp(p))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = run_sort(p, rows, B, 1, p->d_srt, st))) return rc;
    if ((rc = vjp_from_gradient(p, rows, B, (const float2 *)s, (const float2 *)g, eta, tau, (const float2 *)sbar_next,
                                (float2 *)sbar, eta_bar, tau_bar, st)))
        return rc;
    return ok();
}

// ------------------------------------------------------------------------------------------
// Autotuner: time the two tile kernels over candidate launch shapes (row splits, i.e. minibatch
// rows per work-group, and 8 or 16 waves per work-group) and keep the fastest per kernel;
// results are cached in a small JSON file.
// ------------------------------------------------------------------------------------------
static std::string tune_key(const spgm_plan *p, int B) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    std::ostringstream k;
    k << arch << "|phase" << p->phase_mode << "|T" << p->geo.T << "|R" << p->geo.R << "|F" << p->geo.F << "|grid"
      << p->geo.nx << "x" << p->geo.ny << "x" << p->geo.nz << "|B" << B;
    return k.str();
}

// The cache is a flat JSON object {"key": [fwd_splits, adj_splits, fwd_ms, adj_ms, fwd_waves,
// adj_waves], ...}; entries without the last two use the plan's default waves per work-group.
static std::map<std::string, std::vector<double>> read_cache(const std::string &path) {
    std::map<std::string, std::vector<double>> out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t i = 0;
    while ((i = t.find('"', i)) != std::string::npos) {
        const size_t j = t.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = t.substr(i + 1, j - i - 1);
        const size_t a = t.find('[', j), b = t.find(']', j);
        if (a == std::string::npos || b == std::string::npos) break;
        std::vector<double> v;
        std::stringstream vs(t.substr(a + 1, b - a - 1));
        std::string item;
        while (std::getline(vs, item, ',')) v.push_back(std::atof(item.c_str()));
        out[key] = v;
        i = b + 1;
    }
    return out;
}

static void write_cache(const std::string &path, const std::map<std::string, std::vector<double>> &c) {
    std::ofstream f(path + ".tmp");
    if (!f) return;
    f << "{\n";
    size_t n = 0;
    for (const auto &kv : c) {
        f << "  \"" << kv.first << "\": [";
        for (size_t i = 0; i < kv.second.size(); ++i) f << (i ? ", " : "") << kv.second[i];
        f << "]" << (++n < c.size() ? "," : "") << "\n";
    }
    f << "}\n";
    f.close();
    std::rename((path + ".tmp").c_str(), path.c_str());
}

int spgm_plan_autotune(spgm_plan *p, int32_t B, const char *cache_path, int32_t *fwd_out, int32_t *adj_out) {
    if (!p) return fail(SPGM_E_INVALID, "spgm_plan_autotune: plan is NULL");
    if (B < 1 || B > kMaxB) return fail(SPGM_E_INVALID, "spgm_plan_autotune: B=%d outside [1, %d]", B, kMaxB);
    DeviceGuard guard(p->device);
    // The timing runs on a stream of its own and rewrites the plan's workspace: work queued
    // earlier on any stream may still use it.
    if (hipDeviceSynchronize() != hipSuccess) return fail(SPGM_E_DEVICE, "spgm_plan_autotune: device error");
    std::string path = cache_path ? cache_path : p->tune_cache;
    if (path.empty() && std::getenv("SPGM_TUNE_CACHE")) path = std::getenv("SPGM_TUNE_CACHE");
    const std::string key = tune_key(p, B);
    std::map<std::string, std::vector<double>> cache;
    if (!path.empty()) cache = read_cache(path);
    const auto hit = cache.find(key);
    auto waves_ok = [p](int w) { return w == 8 || (w == 16 && tile_lds(p->geo, 16) <= (size_t)kMaxLds); };
    if (hit != cache.end() && hit->second.size() >= 2) {
        const int fw = hit->second.size() >= 6 ? (int)hit->second[4] : p->tile_waves;
        const int aw = hit->second.size() >= 6 ? (int)hit->second[5] : p->tile_waves;
        p->tuned[B] = {TileShape{std::max(1, std::min((int)hit->second[0], max_splits(B))), waves_ok(fw) ? fw : 8},
                       TileShape{std::max(1, std::min((int)hit->second[1], max_splits(B))), waves_ok(aw) ? aw : 8}};
    } else {
        // candidates: 1, 2, 3, 4, 6, 8, 12, 16, ... rows per work-group >= 64
        std::vector<int> cand;
        for (int c = 1; c <= max_splits(B); c = (c < 4 ? c + 1 : c + c / 2)) cand.push_back(c);
        if (cand.back() != max_splits(B)) cand.push_back(max_splits(B));
        if (cand.size() > 10) cand.erase(cand.begin() + 9, cand.end() - 1);
        // timing inputs: uniform pseudo-random rows (xorshift) and a random vector
        std::vector<int32_t> hrows(B);
        uint64_t x = 0x9E3779B97F4A7C15ull ^ (uint64_t)B;
        for (int i = 0; i < B; ++i) {
            x ^= x << 13;
            x ^= x >> 7;
            x ^= x << 17;
            hrows[i] = (int32_t)(x % (uint64_t)p->M);
        }
        std::vector<float2> hs(p->N);
        for (int64_t n = 0; n < p->N; ++n) {
            x ^= x << 13;
            x ^= x >> 7;
            x ^= x << 17;
            hs[n] = make_float2((float)((x >> 11) % 2001) / 1000.f - 1.f, (float)((x >> 33) % 2001) / 1000.f - 1.f);
        }
        int32_t *drows = nullptr;
        float2 *ds = nullptr;
        hipStream_t st = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        int rc = SPGM_OK;
        const int max_c = cand.back();
        if (hipMalloc(&drows, sizeof(int32_t) * B) != hipSuccess || hipMalloc(&ds, sizeof(float2) * p->N) != hipSuccess ||
            hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
            hipEventCreate(&e1) != hipSuccess)
            rc = fail(SPGM_E_NOMEM, "spgm_plan_autotune: allocation failed");
        if (!rc && (hipMemcpy(drows, hrows.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice) != hipSuccess ||
                    hipMemcpy(ds, hs.data(), sizeof(float2) * p->N, hipMemcpyHostToDevice) != hipSuccess))
            rc = fail(SPGM_E_DEVICE, "spgm_plan_autotune: copy failed");
        // size the workspace for the largest candidate
        if (!rc) {
            p->tuned[B] = {TileShape{max_c, 8}, TileShape{max_c, 8}};
            rc = ensure_workspace(p, B);
        }
        if (!rc) rc = run_sort(p, drows, B, 1, p->d_srt, st);
        double best_f = 1e30, best_a = 1e30;
        TileShape bf{1, 8}, ba{1, 8};
        const bool timing = p->timing;
        p->timing = false;
        std::vector<TileShape> shapes;
        for (int w : {8, 16})
            if (waves_ok(w))
                for (int c : cand) shapes.push_back(TileShape{c, w});
        for (size_t ci = 0; !rc && ci < shapes.size(); ++ci) {
            p->tuned[B] = {shapes[ci], shapes[ci]};
            for (int which = 0; which < 2 && !rc; ++which) {
                float best = 1e30f;
                for (int rep = 0; rep < 4 && !rc; ++rep) {
                    if (hipEventRecord(e0, st) != hipSuccess) {
                        rc = fail(SPGM_E_DEVICE, "spgm_plan_autotune: event record failed");
                        break;
                    }
                    rc = which == 0 ? run_forward_partials(p, p->d_srt, ds, B, st) : run_adjoint_partials(p, p->d_srt, B, st);
                    float ms = 0.f;
                    if (!rc && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                        rc = fail(SPGM_E_DEVICE, "spgm_plan_autotune: timing failed");
                    if (!rc && rep > 0) best = std::min(best, ms);  // first launch warms up
                }
                if (which == 0 && best < best_f) {
                    best_f = best;
                    bf = shapes[ci];
                }
                if (which == 1 && best < best_a) {
                    best_a = best;
                    ba = shapes[ci];
                }
            }
        }
        p->timing = timing;
        hipFree(drows);
        hipFree(ds);
        if (st) hipStreamDestroy(st);
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        if (rc) {
            p->tuned.erase(B);
            return rc;
        }
        p->tuned[B] = {bf, ba};
        if (!path.empty()) {
            cache[key] = {(double)bf.splits, (double)ba.splits, best_f, best_a, (double)bf.waves, (double)ba.waves};
            write_cache(path, cache);
        }
    }
    int rc;
    if ((rc = ensure_workspace(p, B))) return rc;
    drop_graph(p);  // launch shapes changed
    if (fwd_out) *fwd_out = p->tuned[B].first.splits;
    if (adj_out) *adj_out = p->tuned[B].second.splits;
    return ok();
}

// ------------------------------------------------------------------------------------------
// Seeded minibatch generator.  SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014): the state advances by the golden-ratio increment and each
// output is the new state through the published 64-bit finaliser.  Iteration k of a solve takes
// outputs k 2^32 + 1, k 2^32 + 2, ... of the sequence seeded with `seed`, so its draws do not
// depend on how the iterations are split over calls.  A partial Fisher-Yates shuffle of
// 0 .. n-1 turns them into m distinct indices: draw j swaps position j with position
// j + floor(hi32(u_j) (n - j) / 2^32) and index j is what position j then holds.
// ------------------------------------------------------------------------------------------
extern "C++" {
struct SplitMix64 {
    uint64_t state;
    uint64_t next() {
        state += 0x9E3779B97F4A7C15ull;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
};

SplitMix64 iteration_stream(uint64_t seed, int64_t k) {
    return SplitMix64{seed + (uint64_t)k * (0x9E3779B97F4A7C15ull << 32)};
}

// m distinct indices of 0 .. n-1 into out; perm holds the identity on entry and on return
// (the positions a call swaps are reset, so a call costs O(m) however large n is).
void fisher_yates(SplitMix64 &gen, int64_t n, int m, int32_t *out, std::vector<int32_t> &perm,
                  std::vector<int64_t> &touched) {
    touched.clear();
    for (int j = 0; j < m; ++j) {
        const uint64_t u = gen.next();
        const int64_t r = j + (int64_t)(((u >> 32) * (uint64_t)(n - j)) >> 32);
        std::swap(perm[j], perm[r]);
        touched.push_back(r);
        out[j] = perm[j];
    }
    for (int64_t r : touched) perm[r] = (int32_t)r;
    for (int j = 0; j < m; ++j) perm[j] = j;
}
}  // extern "C++"

int spgm_rows_generate(uint64_t seed, int32_t start_iter, int32_t iters, int64_t M, int32_t B, int32_t *rows) {
    if (!rows || iters < 0 || start_iter < 0) return fail(SPGM_E_INVALID, "spgm_rows_generate: bad arguments");
    if (M < 1 || M > INT32_MAX || B < 1 || B > M)
        return fail(SPGM_E_INVALID, "spgm_rows_generate: need 1 <= B <= M < 2^31 (B=%d, M=%lld)", B, (long long)M);
    std::vector<int32_t> perm(M);
    for (int64_t i = 0; i < M; ++i) perm[i] = (int32_t)i;
    std::vector<int64_t> touched;
    for (int32_t i = 0; i < iters; ++i) {
        SplitMix64 gen = iteration_stream(seed, (int64_t)start_iter + i);
        fisher_yates(gen, M, B, rows + (size_t)i * B, perm, touched);
    }
    return ok();
}

int spgm_subsets_generate(uint64_t seed, int32_t start_iter, int32_t iters, int32_t F, int32_t T, int32_t R,
                          int32_t nf, int32_t nt, int32_t nr, int32_t *f_idx, int32_t *t_idx, int32_t *r_idx) {
    if (!f_idx || !t_idx || !r_idx || iters < 0 || start_iter < 0)
        return fail(SPGM_E_INVALID, "spgm_subsets_generate: bad arguments");
    if (nf < 1 || nf > F || nt < 1 || nt > T || nr < 1 || nr > R)
        return fail(SPGM_E_INVALID, "spgm_subsets_generate: need 1 <= nf <= F, 1 <= nt <= T, 1 <= nr <= R");
    std::vector<int32_t> pf(F), pt(T), pr(R);
    for (int i = 0; i < F; ++i) pf[i] = i;
    for (int i = 0; i < T; ++i) pt[i] = i;
    for (int i = 0; i < R; ++i) pr[i] = i;
    std::vector<int64_t> touched;
    for (int32_t i = 0; i < iters; ++i) {
        SplitMix64 gen = iteration_stream(seed, (int64_t)start_iter + i);
        fisher_yates(gen, F, nf, f_idx + (size_t)i * nf, pf, touched);
        fisher_yates(gen, T, nt, t_idx + (size_t)i * nt, pt, touched);
        fisher_yates(gen, R, nr, r_idx + (size_t)i * nr, pr, touched);
    }
    return ok();
}

int spgm_solve_opts_init(spgm_solve_opts *o) {
    if (!o) return fail(SPGM_E_INVALID, "spgm_solve_opts_init: opts is NULL");
    std::memset(o, 0, sizeof(*o));
    o->check_every = 50;
    return ok();
}

extern "C++" {
// Device buffer for `n` generated values and the two pinned staging buffers.
static int gen_buffers(spgm_plan *p, size_t n) {
    int rc;
    if ((rc = grow_buf(p->d_gen, p->gen_cap, n))) return rc;
    if (n > p->h_gen_cap) {
        for (int i = 0; i < 2; ++i) {
            if (p->gen_ev[i]) hipEventSynchronize(p->gen_ev[i]);
            if (p->h_gen[i]) hipHostFree(p->h_gen[i]);
            p->h_gen[i] = nullptr;
        }
        p->h_gen_cap = 0;
        for (int i = 0; i < 2; ++i)
            if (hipHostMalloc((void **)&p->h_gen[i], sizeof(int32_t) * n, hipHostMallocDefault) != hipSuccess)
                return fail(SPGM_E_NOMEM, "spgm_solve_ex: pinned staging allocation failed");
        p->h_gen_cap = n;
    }
    for (int i = 0; i < 2; ++i)
        if (!p->gen_ev[i] && hipEventCreateWithFlags(&p->gen_ev[i], hipEventDisableTiming) != hipSuccess)
            return fail(SPGM_E_NOMEM, "spgm_solve_ex: event creation failed");
    return SPGM_OK;
}
}  // extern "C++"

int spgm_solve_ex(spgm_plan *p, const void *y, void *s, const spgm_solve_opts *o, void *stream) {
    if (!p || !o) return fail(SPGM_E_INVALID, "spgm_solve_ex: plan and opts must be non-NULL");
    if (o->iters_done) *o->iters_done = 0;
    if (o->iters < 0 || o->start_iter < 0) return fail(SPGM_E_INVALID, "spgm_solve_ex: iters and start_iter must be >= 0");
    if (!(o->eta > 0.0) || !std::isfinite(o->eta) || !(o->lambda >= 0.0) || !std::isfinite(o->lambda))
        return fail(SPGM_E_INVALID, "spgm_solve_ex: need eta > 0 and lambda >= 0, both finite");
    if (o->sampling != 0 && o->sampling != 1) return fail(SPGM_E_INVALID, "spgm_solve_ex: unknown sampling %d", o->sampling);
    const float eta = (float)o->eta, alpha = (float)(o->lambda * o->eta);
    hipStream_t st = (hipStream_t)stream;
    if (o->iters == 0) return ok();
    DeviceGuard guard(p->device);
    int rc;
    if (o->sampling == 1) {
        // structured minibatches from the generator: fixed iterations, eager launches
        if (o->rows_d) return fail(SPGM_E_INVALID, "spgm_solve_ex: structured sampling draws its own subsets (rows_d must be NULL)");
        if (o->tol > 0.0 || o->use_graph)
            return fail(SPGM_E_UNSUPPORTED, "spgm_solve_ex: structured sampling runs fixed iterations without a graph");
        const int nf = o->nf, nt = o->nt, nr = o->nr;
        if (nf < 1 || nf > p->geo.F || nt < 1 || nt > p->geo.T || nr < 1 || nr > p->geo.R)
            return fail(SPGM_E_INVALID, "spgm_solve_ex: need 1 <= nf <= F, 1 <= nt <= T, 1 <= nr <= R");
        const int per = std::max(1, std::min(o->iters, (1 << 20) / (nf + nt + nr)));
        if ((rc = gen_buffers(p, (size_t)per * (nf + nt + nr)))) return rc;
        for (int i0 = 0, c = 0; i0 < o->iters; i0 += per, ++c) {
            const int cnt = std::min(per, o->iters - i0);
            int32_t *h = p->h_gen[c & 1];
            if (hipEventSynchronize(p->gen_ev[c & 1]) != hipSuccess) return fail(SPGM_E_DEVICE, "spgm_solve_ex: device error");
            if ((rc = spgm_subsets_generate(o->seed, o->start_iter + i0, cnt, p->geo.F, p->geo.T, p->geo.R, nf, nt, nr,
                                            h, h + (size_t)cnt * nf, h + (size_t)cnt * (nf + nt))))
                return rc;
            const size_t n = (size_t)cnt * (nf + nt + nr);
            if (hipMemcpyAsync(p->d_gen, h, sizeof(int32_t) * n, hipMemcpyHostToDevice, st) != hipSuccess ||
                hipEventRecord(p->gen_ev[c & 1], st) != hipSuccess)
                return fail(SPGM_E_DEVICE, "spgm_solve_ex: upload failed");
            if ((rc = spgm_solve_structured(p, p->d_gen, nf, p->d_gen + (size_t)cnt * nf, nt,
                                            p->d_gen + (size_t)cnt * (nf + nt), nr, cnt, y, s, eta, alpha, stream)))
                return rc;
            if (o->iters_done) *o->iters_done = i0 + cnt;
        }
        return ok();
    }
    const int B = o->B;
    if (B < 1 || B > kMaxB) return fail(SPGM_E_INVALID, "spgm_solve_ex: B=%d outside [1, %d]", B, kMaxB);
    auto run = [&](const int32_t *rows, int cnt, int *done) {
        *done = cnt;
        if (o->tol > 0.0)
            return spgm_solve_tol(p, rows, cnt, B, y, s, eta, alpha, o->tol, std::max(1, o->check_every), o->use_graph,
                                  done, nullptr, stream);
        return o->use_graph ? spgm_solve_graph(p, rows, cnt, B, y, s, eta, alpha, stream)
                            : spgm_solve(p, rows, cnt, B, y, s, eta, alpha, stream);
    };
    if (o->rows_d) {
        int done = 0;
        rc = run(o->rows_d, o->iters, &done);
        if (o->iters_done) *o->iters_done = done;
        return rc ? rc : ok();
    }
    if (B > p->M) return fail(SPGM_E_INVALID, "spgm_solve_ex: generated minibatches need B <= M (%d > %lld)", B, (long long)p->M);
    const int per = std::max(1, std::min(o->iters, (1 << 22) / B));
    if ((rc = gen_buffers(p, (size_t)per * B))) return rc;
    for (int i0 = 0, c = 0; i0 < o->iters; i0 += per, ++c) {
        const int cnt = std::min(per, o->iters - i0);
        int32_t *h = p->h_gen[c & 1];
        // the staging buffer's previous upload has finished before it is refilled
        if (hipEventSynchronize(p->gen_ev[c & 1]) != hipSuccess) return fail(SPGM_E_DEVICE, "spgm_solve_ex: device error");
        if ((rc = spgm_rows_generate(o->seed, o->start_iter + i0, cnt, p->M, B, h))) return rc;
        if (hipMemcpyAsync(p->d_gen, h, sizeof(int32_t) * (size_t)cnt * B, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipEventRecord(p->gen_ev[c & 1], st) != hipSuccess)
            return fail(SPGM_E_DEVICE, "spgm_solve_ex: upload failed");
        int done = 0;
        rc = run(p->d_gen, cnt, &done);
        if (o->iters_done) *o->iters_done = i0 + done;
        if (rc) return rc;
        if (done < cnt) break;  // termination rule met
    }
    return ok();
}

// ------------------------------------------------------------------------------------------
// Autotuner of the shared-geometry batch kernels: forward (row tiles per wave, bricks per
// work-group, waves and z slices per work-group) and adjoint (row splits, staged rows per round)
// timed separately on pseudo-random rows and right-hand sides, keyed in the same cache.
// ------------------------------------------------------------------------------------------
extern "C++" {
static std::vector<std::array<int, 4>> mm_fwd_candidates(const spgm_plan *p, int B) {
    std::vector<std::array<int, 4>> out;
    for (int nrt = 1; nrt <= 4; ++nrt)
        for (const auto &wz : {std::array<int, 2>{kWaves, kBZ}, std::array<int, 2>{4, 2}}) {
            MMFwdCfg c;
            if (!mm_fwd_shape(p, B, nrt, 0, wz[0], wz[1], c)) continue;
            for (int bpw : {std::max(1, c.bpw / 2), c.bpw, 2 * c.bpw}) {
                MMFwdCfg d;
                if (!mm_fwd_shape(p, B, nrt, bpw, wz[0], wz[1], d)) continue;
                const std::array<int, 4> v{nrt, d.bpw, wz[0], wz[1]};
                if (std::find(out.begin(), out.end(), v) == out.end()) out.push_back(v);
            }
        }
    return out;
}

static std::vector<std::array<int, 2>> mm_adj_candidates(const spgm_plan *p, int B) {
    std::vector<std::array<int, 2>> out;
    const int d = mm_default_adj_splits(p, B);
    for (int sp : {d, 2 * d, 4 * d})
        for (int stage : {0, 4 * kMMStage, kMMStage}) {
            MMAdjCfg c;
            if (!mm_adj_shape(p, B, sp, stage, c)) continue;
            const std::array<int, 2> v{c.splits, c.stage};
            if (std::find(out.begin(), out.end(), v) == out.end()) out.push_back(v);
        }
    return out;
}

template <int PREC>
static int mm_tune_time(spgm_plan *p, int B, const float2 *S, const float2 *R, float2 *G, hipStream_t st,
                        hipEvent_t e0, hipEvent_t e1, std::array<int, 4> &bf, std::array<int, 2> &ba, double &tf,
                        double &ta) {
    int rc = SPGM_OK;
    auto timed = [&](auto &&launch, float &best) {
        best = 1e30f;
        for (int rep = 0; rep < 4 && !rc; ++rep) {
            if (hipEventRecord(e0, st) != hipSuccess) return (rc = fail(SPGM_E_DEVICE, "autotune: event failed"));
            if ((rc = launch())) return rc;
            float ms = 0.f;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                return (rc = fail(SPGM_E_DEVICE, "autotune: timing failed"));
            if (rep > 0) best = std::min(best, ms);  // the first launch warms up
        }
        return rc;
    };
    tf = ta = 1e30;
    bool packed = false;
    for (const auto &v : mm_fwd_candidates(p, B)) {
        p->mm_fwd_tuned[B] = v;
        if ((rc = ensure_mm(p, B))) return rc;
        const MMFwdCfg fc = mm_fwd_cfg(p, B);
        if (!packed) {
            if ((rc = mm_forward_pass<PREC>(p, fc, p->d_srt, B, S, kMMCols, 0, kMMCols, st, true))) return rc;
            packed = true;
        }
        float ms;
        if (timed([&] { return mm_forward_pass<PREC>(p, fc, p->d_srt, B, S, kMMCols, 0, kMMCols, st, false); }, ms))
            return rc;
        if (ms < tf) {
            tf = ms;
            bf = v;
        }
    }
    p->mm_fwd_tuned[B] = bf;
    const int quads = ((B + 7) & ~7) / 4;
    k_mm_pack_r<PREC><<<(quads + 7) / 8, 256, 0, st>>>(p->geo, p->d_srt, B, R, kMMCols, 0, kMMCols, p->d_mm_r);
    if ((rc = launch_check("autotune pack"))) return rc;
    for (const auto &v : mm_adj_candidates(p, B)) {
        p->mm_adj_tuned[B] = v;
        if ((rc = ensure_mm(p, B))) return rc;
        const MMAdjCfg ac = mm_adj_cfg(p, B);
        const MMAdjOut out{0, kMMCols, kMMCols, G, nullptr, 0.f, 0.f, nullptr};
        float ms;
        if (timed([&] { return mm_adjoint_pass<PREC>(p, ac, p->d_srt, B, out, st); }, ms)) return rc;
        if (ms < ta) {
            ta = ms;
            ba = v;
        }
    }
    p->mm_adj_tuned[B] = ba;
    return rc;
}

}  // extern "C++"

int spgm_plan_autotune_batched(spgm_plan *p, int32_t B, int32_t prec, const char *cache_path, int32_t *shape) {
    if (!p) return fail(SPGM_E_INVALID, "spgm_plan_autotune_batched: plan is NULL");
    if (B < 1 || B > kMaxB) return fail(SPGM_E_INVALID, "spgm_plan_autotune_batched: B=%d outside [1, %d]", B, kMaxB);
    if (prec != SPGM_MM_BF16 && prec != SPGM_MM_FP16)
        return fail(SPGM_E_INVALID, "spgm_plan_autotune_batched: unknown precision %d", prec);
    if (p->phase_mode != SPGM_PHASE_COMP32)
        return fail(SPGM_E_UNSUPPORTED, "spgm_plan_autotune_batched: needs a plan created with SPGM_PHASE_COMP32");
    DeviceGuard guard(p->device);
    if (hipDeviceSynchronize() != hipSuccess) return fail(SPGM_E_DEVICE, "spgm_plan_autotune_batched: device error");
    std::string path = cache_path ? cache_path : p->tune_cache;
    if (path.empty() && std::getenv("SPGM_TUNE_CACHE")) path = std::getenv("SPGM_TUNE_CACHE");
    const std::string key = tune_key(p, B) + "|mm" + std::to_string(prec);
    std::map<std::string, std::vector<double>> cache;
    if (!path.empty()) cache = read_cache(path);
    const auto hit = cache.find(key);
    int rc = SPGM_OK;
    if (hit != cache.end() && hit->second.size() >= 6) {
        const auto &v = hit->second;
        p->mm_fwd_tuned[B] = {(int)v[0], (int)v[1], (int)v[2], (int)v[3]};
        p->mm_adj_tuned[B] = {(int)v[4], (int)v[5]};
    } else {
        // timing inputs: uniform pseudo-random rows (xorshift) and right-hand sides
        uint64_t x = 0x2545F4914F6CDD1Dull ^ (uint64_t)B;
        auto next = [&x]() {
            x ^= x << 13;
            x ^= x >> 7;
            x ^= x << 17;
            return x;
        };
        std::vector<int32_t> hrows(B);
        for (int i = 0; i < B; ++i) hrows[i] = (int32_t)(next() % (uint64_t)p->M);
        const size_t ns = (size_t)p->N * kMMCols, nr = (size_t)B * kMMCols;
        std::vector<float2> hv(std::max(ns, nr));
        for (auto &v : hv) {
            const uint64_t r = next();
            v = make_float2((float)((r >> 11) % 2001) / 1000.f - 1.f, (float)((r >> 33) % 2001) / 1000.f - 1.f);
        }
        int32_t *drows = nullptr;
        float2 *dS = nullptr, *dR = nullptr, *dG = nullptr;
        hipStream_t st = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipMalloc(&drows, sizeof(int32_t) * B) != hipSuccess || hipMalloc(&dS, sizeof(float2) * ns) != hipSuccess ||
            hipMalloc(&dR, sizeof(float2) * nr) != hipSuccess || hipMalloc(&dG, sizeof(float2) * ns) != hipSuccess ||
            hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
            hipEventCreate(&e1) != hipSuccess)
            rc = fail(SPGM_E_NOMEM, "spgm_plan_autotune_batched: allocation failed");
        if (!rc && (hipMemcpy(drows, hrows.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice) != hipSuccess ||
                    hipMemcpy(dS, hv.data(), sizeof(float2) * ns, hipMemcpyHostToDevice) != hipSuccess ||
                    hipMemcpy(dR, hv.data(), sizeof(float2) * nr, hipMemcpyHostToDevice) != hipSuccess))
            rc = fail(SPGM_E_DEVICE, "spgm_plan_autotune_batched: copy failed");
        if (!rc) rc = ensure_workspace(p, B);
        if (!rc) rc = run_sort(p, drows, B, 1, p->d_srt, st);
        std::array<int, 4> bf{};
        std::array<int, 2> ba{};
        double tf = 0.0, ta = 0.0;
        const bool timing = p->timing;
        p->timing = false;
        if (!rc)
            rc = prec == SPGM_MM_FP16 ? mm_tune_time<SPGM_MM_FP16>(p, B, dS, dR, dG, st, e0, e1, bf, ba, tf, ta)
                                      : mm_tune_time<SPGM_MM_BF16>(p, B, dS, dR, dG, st, e0, e1, bf, ba, tf, ta);
        p->timing = timing;
        if (st) hipStreamSynchronize(st);
        hipFree(drows);
        hipFree(dS);
        hipFree(dR);
        hipFree(dG);
        if (st) hipStreamDestroy(st);
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        if (rc) {
            p->mm_fwd_tuned.erase(B);
            p->mm_adj_tuned.erase(B);
            return rc;
        }
        if (!path.empty()) {
            cache[key] = {(double)bf[0], (double)bf[1], (double)bf[2], (double)bf[3], (double)ba[0], (double)ba[1],
                          tf, ta};
            write_cache(path, cache);
        }
    }
    if (mm_fwd_cfg(p, B).lds > (size_t)kMaxLds || mm_adj_cfg(p, B).lds > (size_t)kMaxLds)
        return fail(SPGM_E_UNSUPPORTED, "spgm_plan_autotune_batched: brick tables exceed LDS");
    if ((rc = ensure_mm(p, B))) return rc;
    return spgm_plan_batched_shape(p, B, shape);
}

int spgm_plan_batched_shape(const spgm_plan *p, int32_t B, int32_t *shape) {
    if (!p || !shape) return fail(SPGM_E_INVALID, "spgm_plan_batched_shape: plan and shape must be non-NULL");
    if (B < 1 || B > kMaxB) return fail(SPGM_E_INVALID, "spgm_plan_batched_shape: B=%d outside [1, %d]", B, kMaxB);
    const MMFwdCfg f = mm_fwd_cfg(p, B);
    const MMAdjCfg a = mm_adj_cfg(p, B);
    const int32_t v[7] = {f.nrt, f.bpw, f.waves, f.zs, a.splits, a.stage, f.rows_form ? 1 : 0};
    std::memcpy(shape, v, sizeof(v));
    return ok();
}

int spgm_plan_batched_candidates(const spgm_plan *p, int32_t B, int32_t *fwd, int32_t fwd_cap, int32_t *n_fwd,
                                 int32_t *adj, int32_t adj_cap, int32_t *n_adj) {
    if (!p || !n_fwd || !n_adj) return fail(SPGM_E_INVALID, "spgm_plan_batched_candidates: NULL argument");
    if (B < 1 || B > kMaxB) return fail(SPGM_E_INVALID, "spgm_plan_batched_candidates: B=%d outside [1, %d]", B, kMaxB);
    const auto f = mm_fwd_candidates(p, B);
    const auto a = mm_adj_candidates(p, B);
    *n_fwd = (int32_t)f.size();
    *n_adj = (int32_t)a.size();
    for (int i = 0; fwd && i < std::min((int)f.size(), fwd_cap); ++i)
        for (int k = 0; k < 4; ++k) fwd[4 * i + k] = f[i][k];
    for (int i = 0; adj && i < std::min((int)a.size(), adj_cap); ++i)
        for (int k = 0; k < 2; ++k) adj[2 * i + k] = a[i][k];
    return ok();
}

// ------------------------------------------------------------------------------------------
// Autotuner of the structured-minibatch kernels: the small-register instances (8 items per
// thread, for nt + nr <= 32 and nt <= 16) or the general ones (16 items), timed on the forward
// and adjoint kernels of subsets of the first nf frequencies, nt transmitters and nr receivers.
// ------------------------------------------------------------------------------------------
int spgm_plan_autotune_structured(spgm_plan *p, int32_t nf, int32_t nt, int32_t nr, const char *cache_path,
                                  int32_t *items) {
    if (!p) return fail(SPGM_E_INVALID, "spgm_plan_autotune_structured: plan is NULL");
    if (nf < 1 || nt < 1 || nr < 1 || nf > p->geo.F || nt > p->geo.T || nr > p->geo.R)
        return fail(SPGM_E_INVALID, "spgm_plan_autotune_structured: need 1 <= nf <= F, 1 <= nt <= T, 1 <= nr <= R");
    DeviceGuard guard(p->device);
    if (hipDeviceSynchronize() != hipSuccess) return fail(SPGM_E_DEVICE, "spgm_plan_autotune_structured: device error");
    std::vector<int32_t> idx(std::max(nf, std::max(nt, nr)));
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int32_t)i;
    int32_t *d_idx = nullptr;
    if (hipMalloc(&d_idx, sizeof(int32_t) * idx.size()) != hipSuccess)
        return fail(SPGM_E_NOMEM, "spgm_plan_autotune_structured: allocation failed");
    if (hipMemcpy(d_idx, idx.data(), sizeof(int32_t) * idx.size(), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(d_idx);
        return fail(SPGM_E_DEVICE, "spgm_plan_autotune_structured: copy failed");
    }
    const SFArgs a{d_idx, d_idx, d_idx, nf, nt, nr, nf * nt * nr};
    int rc = sf_check(p, a, "spgm_plan_autotune_structured");
    std::string path = cache_path ? cache_path : p->tune_cache;
    if (path.empty() && std::getenv("SPGM_TUNE_CACHE")) path = std::getenv("SPGM_TUNE_CACHE");
    std::ostringstream ks;
    ks << tune_key(p, a.B) << "|sf|nf" << nf << "|nt" << nt << "|nr" << nr;
    const std::string key = ks.str();
    std::map<std::string, std::vector<double>> cache;
    if (!rc && !path.empty()) cache = read_cache(path);
    const auto hit = cache.find(key);
    const std::array<int, 3> sk{nf, nt, nr};
    if (!rc && hit != cache.end() && !hit->second.empty()) {
        const int v = (int)hit->second[0];
        p->sf_tuned[sk] = (v == kSFItemsSmall && sf_small_ok(a)) ? kSFItemsSmall : kSFItems;
    } else if (!rc) {
        float2 *ds = nullptr;
        hipStream_t st = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipMalloc(&ds, sizeof(float2) * p->N) != hipSuccess ||
            hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
            hipEventCreate(&e1) != hipSuccess)
            rc = fail(SPGM_E_NOMEM, "spgm_plan_autotune_structured: allocation failed");
        if (!rc && hipMemsetAsync(ds, 0, sizeof(float2) * p->N, st) != hipSuccess)
            rc = fail(SPGM_E_DEVICE, "spgm_plan_autotune_structured: fill failed");
        if (!rc) rc = sf_prepare(p, a, st);
        if (!rc && hipMemsetAsync(p->d_rs, 0, sizeof(float2) * a.B, st) != hipSuccess)
            rc = fail(SPGM_E_DEVICE, "spgm_plan_autotune_structured: fill failed");
        const bool timing = p->timing;
        p->timing = false;
        double best = 1e30;
        int best_items = kSFItems;
        for (int cand : {kSFItemsSmall, kSFItems}) {
            if (rc) break;
            if (cand == kSFItemsSmall && !sf_small_ok(a)) continue;
            p->sf_tuned[sk] = cand;
            float tbest = 1e30f;
            for (int rep = 0; rep < 4 && !rc; ++rep) {
                float ms = 0.f;
                if (hipEventRecord(e0, st) != hipSuccess) rc = fail(SPGM_E_DEVICE, "autotune: event failed");
                if (!rc) rc = sf_forward_partials(p, a, ds, st);
                if (!rc) rc = sf_adjoint_partials(p, a, st);
                if (!rc && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    rc = fail(SPGM_E_DEVICE, "spgm_plan_autotune_structured: timing failed");
                if (!rc && rep > 0) tbest = std::min(tbest, ms);
            }
            if (!rc && tbest < best) {
                best = tbest;
                best_items = cand;
            }
        }
        p->timing = timing;
        if (st) hipStreamSynchronize(st);
        hipFree(ds);
        if (st) hipStreamDestroy(st);
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        if (rc) {
            p->sf_tuned.erase(sk);
        } else {
            p->sf_tuned[sk] = best_items;
            if (!path.empty()) {
                cache[key] = {(double)best_items, best};
                write_cache(path, cache);
            }
        }
    }
    hipFree(d_idx);
    if (rc) return rc;
    return spgm_plan_structured_shape(p, nf, nt, nr, items);
}

int spgm_plan_structured_shape(const spgm_plan *p, int32_t nf, int32_t nt, int32_t nr, int32_t *items) {
    if (!p || !items) return fail(SPGM_E_INVALID, "spgm_plan_structured_shape: plan and items must be non-NULL");
    const SFArgs a{nullptr, nullptr, nullptr, nf, nt, nr, nf * nt * nr};
    *items = sf_small(p, a) ? kSFItemsSmall : kSFItems;
    return ok();
}

// ------------------------------------------------------------------------------------------
// Ragged batches
// ------------------------------------------------------------------------------------------
int spgm_batch_create(spgm_batch **out, const spgm_geometry *geoms, int32_t n, int32_t phase_mode) {
    if (!out) return fail(SPGM_E_INVALID, "spgm_batch_create: out is NULL");
    *out = nullptr;
    if (!geoms || n < 1) return fail(SPGM_E_INVALID, "spgm_batch_create: need n >= 1 geometries");
    spgm_batch *b = new spgm_batch();
    b->phase_mode = phase_mode;
    for (int i = 0; i < n; ++i) {
        spgm_plan *p = nullptr;
        const int rc = spgm_plan_create(&p, geoms + i, phase_mode);
        if (rc) {
            const std::string msg = g_last_error;
            spgm_batch_destroy(b);
            return fail(rc, "spgm_batch_create: scene %d: %s", i, msg.c_str());
        }
        b->plans.push_back(p);
    }
    b->device = b->plans[0]->device;
    DeviceGuard guard(b->device);
    if (hipMalloc(&b->d_status, sizeof(int)) != hipSuccess || hipMemset(b->d_status, 0, sizeof(int)) != hipSuccess) {
        spgm_batch_destroy(b);
        return fail(SPGM_E_NOMEM, "spgm_batch_create: allocation failed");
    }
    *out = b;
    return ok();
}

int spgm_batch_destroy(spgm_batch *b) {
    if (!b) return ok();
    {
        DeviceGuard guard(b->device);
        hipDeviceSynchronize();
        hipFree(b->d_status);
        hipFree(b->d_scenes);
        hipFree(b->d_items);
        hipFree(b->d_blocks);
        hipFree(b->d_ws);
        if (b->cap_stream) hipStreamDestroy(b->cap_stream);
    }
    for (spgm_plan *p : b->plans) spgm_plan_destroy(p);
    delete b;
    return ok();
}

int spgm_batch_plan(spgm_batch *b, int32_t i, spgm_plan **plan) {
    if (!b || !plan || i < 0 || i >= (int)b->plans.size()) return fail(SPGM_E_INVALID, "spgm_batch_plan: bad argument");
    *plan = b->plans[i];
    return ok();
}

extern "C++" {
template <typename T> static int grow(T *&ptr, size_t &cap, size_t need) {
    if (need <= cap) return SPGM_OK;
    hipFree(ptr);
    ptr = nullptr;
    cap = 0;
    if (hipMalloc(&ptr, sizeof(T) * need) != hipSuccess) return fail(SPGM_E_NOMEM, "spgm_batch: allocation failed");
    cap = need;
    return SPGM_OK;
}
}

static int batch_launches(spgm_batch *b, int iters, int n_items, int grid_items, size_t lds, int max_chunks, int p2,
                          int n_rblocks, int n_cblocks, hipStream_t st) {
    const int n = (int)b->plans.size();
    const int mode = b->phase_mode;
    for (int k = 0; k < iters; ++k) {
        k_sort_scenes<<<dim3(max_chunks, n), kSortThreads, sizeof(unsigned long long) * p2, st>>>(b->d_scenes, k,
                                                                                                 b->d_status);
        if (mode == SPGM_PHASE_F64)
            k_fwd_items<SPGM_PHASE_F64><<<grid_items, kThreads, lds, st>>>(b->d_scenes, b->d_items, n_items);
        else if (mode == SPGM_PHASE_NAIVE32)
            k_fwd_items<SPGM_PHASE_NAIVE32><<<grid_items, kThreads, lds, st>>>(b->d_scenes, b->d_items, n_items);
        else
            k_fwd_items<SPGM_PHASE_COMP32><<<grid_items, kThreads, lds, st>>>(b->d_scenes, b->d_items, n_items);
        k_row_reduce_scenes<<<n_rblocks, 64 * kRedGroups, 0, st>>>(b->d_scenes, b->d_blocks, k);
        if (mode == SPGM_PHASE_F64)
            k_adj_items<SPGM_PHASE_F64><<<grid_items, kThreads, lds, st>>>(b->d_scenes, b->d_items, n_items);
        else if (mode == SPGM_PHASE_NAIVE32)
            k_adj_items<SPGM_PHASE_NAIVE32><<<grid_items, kThreads, lds, st>>>(b->d_scenes, b->d_items, n_items);
        else
            k_adj_items<SPGM_PHASE_COMP32><<<grid_items, kThreads, lds, st>>>(b->d_scenes, b->d_items, n_items);
        k_col_reduce_scenes<<<n_cblocks, 256, 0, st>>>(b->d_scenes, b->d_blocks + n_rblocks);
        int rc;
        if ((rc = launch_check("batch iteration"))) return rc;
    }
    return SPGM_OK;
}

int spgm_batch_solve(spgm_batch *b, int32_t iters, const int32_t *B, const int32_t *const *rows, const void *const *y,
                     void *const *s, const float *eta, const float *alpha, int32_t use_graph, void *stream) {
    if (!b) return fail(SPGM_E_INVALID, "spgm_batch_solve: batch is NULL");
    if (!B || !rows || !y || !s || !eta || !alpha) return fail(SPGM_E_INVALID, "spgm_batch_solve: NULL argument array");
    if (iters < 0) return fail(SPGM_E_INVALID, "spgm_batch_solve: iters must be >= 0");
    const int n = (int)b->plans.size();
    for (int i = 0; i < n; ++i) {
        if (B[i] < 1 || B[i] > kMaxB) return fail(SPGM_E_INVALID, "spgm_batch_solve: scene %d: B=%d out of range", i, B[i]);
        if (!rows[i] || !y[i] || !s[i]) return fail(SPGM_E_INVALID, "spgm_batch_solve: scene %d: NULL pointer", i);
        if (!(std::isfinite(eta[i]) && eta[i] > 0) || !(std::isfinite(alpha[i]) && alpha[i] >= 0))
            return fail(SPGM_E_INVALID, "spgm_batch_solve: scene %d: eta must be > 0 and alpha >= 0", i);
    }
    if (iters == 0) return ok();
    DeviceGuard guard(b->device);
    hipStream_t st = (hipStream_t)stream;
    // The descriptors, work list and workspace below are rewritten on the host: earlier solves
    // queued on the caller's stream may still read them.
    if (hipStreamSynchronize(st) != hipSuccess) return fail(SPGM_E_DEVICE, "spgm_batch_solve: stream error");
    // Layout of the scenes' workspace and the work list.
    std::vector<SceneDev> h(n);
    std::vector<size_t> off(n);
    size_t ws = 0;
    auto take = [&ws](size_t bytes) {
        const size_t o = ws;
        ws += (bytes + 255) / 256 * 256;
        return o;
    };
    struct Item { int4 v; long cost; };
    std::vector<Item> items;
    std::vector<int2> rblocks, cblocks;
    size_t lds = 0;
    int max_chunks = 1, p2 = 2;
    for (int i = 0; i < n; ++i) {
        spgm_plan *p = b->plans[i];
        SceneDev &d = h[i];
        d.geo = p->geo;
        d.B = B[i];
        d.splits = std::max(1, (B[i] + b->rows_per_split - 1) / b->rows_per_split);
        d.rpw = (B[i] + d.splits - 1) / d.splits;
        d.n_tiles = p->n_tiles;
        d.N = (int)p->N;
        d.rows = rows[i];
        d.y = (const float2 *)y[i];
        d.s = (float2 *)s[i];
        d.step = eta[i] / (float)B[i];
        d.alpha = alpha[i];
        off[i] = take(sizeof(int4) * B[i]);
        take(sizeof(float2) * (size_t)d.n_tiles * B[i]);
        take(sizeof(float2) * B[i]);
        take(sizeof(float2) * (size_t)d.splits * d.N);
        for (int t = 0; t < d.n_tiles; ++t)
            for (int sp = 0; sp < d.splits; ++sp) {
                const int rows_here = std::min(d.rpw, B[i] - sp * d.rpw);
                if (rows_here > 0) items.push_back({make_int4(i, t, sp, 0), (long)rows_here});
            }
        for (int r = 0; r < B[i]; r += 64) rblocks.push_back(make_int2(i, r));
        for (int v = 0; v < d.N; v += 256) cblocks.push_back(make_int2(i, v));
        lds = std::max(lds, p->lds_bytes);
        max_chunks = std::max(max_chunks, (B[i] + kSortChunk - 1) / kSortChunk);
        while (p2 < std::min(B[i], kSortChunk)) p2 <<= 1;
    }
    // longest first; ties keep scene/brick order (deterministic)
    std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &c) { return a.cost > c.cost; });
    std::vector<int4> hitems(items.size());
    for (size_t k = 0; k < items.size(); ++k) hitems[k] = items[k].v;
    int rc;
    if ((rc = grow(b->d_ws, b->ws_cap, ws)) || (rc = grow(b->d_scenes, b->scenes_cap, (size_t)n)) ||
        (rc = grow(b->d_items, b->items_cap, hitems.size())) ||
        (rc = grow(b->d_blocks, b->blocks_cap, rblocks.size() + cblocks.size())))
        return rc;
    for (int i = 0; i < n; ++i) {
        SceneDev &d = h[i];
        char *base = b->d_ws + off[i];
        d.srt = (int4 *)base;
        base += ((sizeof(int4) * d.B) + 255) / 256 * 256;
        d.part = (float2 *)base;
        base += ((sizeof(float2) * (size_t)d.n_tiles * d.B) + 255) / 256 * 256;
        d.rs = (float2 *)base;
        base += ((sizeof(float2) * d.B) + 255) / 256 * 256;
        d.gpart = (float2 *)base;
    }
    std::vector<int2> blocks(rblocks);
    blocks.insert(blocks.end(), cblocks.begin(), cblocks.end());
    // descriptors and lists are uploaded synchronously, ahead of any (captured) launch
    if (hipMemcpy(b->d_scenes, h.data(), sizeof(SceneDev) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_items, hitems.data(), sizeof(int4) * hitems.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_blocks, blocks.data(), sizeof(int2) * blocks.size(), hipMemcpyHostToDevice) != hipSuccess)
        return fail(SPGM_E_DEVICE, "spgm_batch_solve: upload failed");
    const void *ik[] = {(const void *)k_fwd_items<SPGM_PHASE_COMP32>, (const void *)k_fwd_items<SPGM_PHASE_F64>,
                        (const void *)k_fwd_items<SPGM_PHASE_NAIVE32>, (const void *)k_adj_items<SPGM_PHASE_COMP32>,
                        (const void *)k_adj_items<SPGM_PHASE_F64>, (const void *)k_adj_items<SPGM_PHASE_NAIVE32>};
    for (const void *k : ik) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void *)k_sort_scenes, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(sizeof(unsigned long long) * kSortChunk));
    hipGetLastError();
    // persistent grid: as many work-groups as fit on the chip at once
    const int per_cu = std::max(1, std::min(2, (int)((160 * 1024) / std::max<size_t>(lds, 1))));
    const int n_items = (int)hitems.size();
    const int fill = b->max_wg > 0 ? b->max_wg : 256 * per_cu;
    const int grid_items = std::max(1, std::min(n_items, fill));
    const int n_rb = (int)rblocks.size(), n_cb = (int)cblocks.size();
    if (!use_graph) {
        if ((rc = batch_launches(b, iters, n_items, grid_items, lds, max_chunks, p2, n_rb, n_cb, st))) return rc;
        return ok();
    }
    if (!b->cap_stream && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return fail(SPGM_E_DEVICE, "spgm_batch_solve: stream creation failed");
    if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(SPGM_E_DEVICE, "spgm_batch_solve: capture failed to start");
    rc = batch_launches(b, iters, n_items, grid_items, lds, max_chunks, p2, n_rb, n_cb, b->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (rc) {
        if (g) hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || !g) return fail(SPGM_E_DEVICE, "spgm_batch_solve: capture failed");
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        hipGraphDestroy(g);
        return fail(SPGM_E_DEVICE, "spgm_batch_solve: graph instantiation failed");
    }
    const hipError_t le = hipGraphLaunch(ex, st);
    hipGraphExecDestroy(ex);  // safe: destruction is deferred until the launch completes
    hipGraphDestroy(g);
    if (le != hipSuccess) return fail(SPGM_E_DEVICE, "spgm_batch_solve: graph launch failed");
    return ok();
}

int spgm_calibrate(int32_t kind, int32_t iters, double *ops_per_s, double *ms) {
    if (kind < 0 || kind > 3) return fail(SPGM_E_INVALID, "spgm_calibrate: kind must be 0..3");
    if (iters < 1 || iters > (1 << 20)) return fail(SPGM_E_INVALID, "spgm_calibrate: iters must be in [1, 2^20]");
    if (!ops_per_s) return fail(SPGM_E_INVALID, "spgm_calibrate: ops_per_s is NULL");
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(SPGM_E_DEVICE, "spgm_calibrate: no HIP device");
    const int grid = prop.multiProcessorCount * 8;
    float *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipMalloc(&out, sizeof(float) * grid) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        hipFree(out);
        if (e0) hipEventDestroy(e0);
        return fail(SPGM_E_NOMEM, "spgm_calibrate: allocation failed");
    }
    auto launch = [&](int n) {
        switch (kind) {
        case 0: k_probe_rate<0><<<grid, 256>>>(out, n, 0.5f); break;
        case 1: k_probe_rate<1><<<grid, 256>>>(out, n, 0.5f); break;
        case 2: k_probe_rate<2><<<grid, 256>>>(out, n, 0.5f); break;
        default: k_probe_rate<3><<<grid, 256>>>(out, n, 0.5f);
        }
    };
    launch(iters);  // warm-up
    hipEventRecord(e0, nullptr);
    launch(iters);
    hipEventRecord(e1, nullptr);
    float t = 0.f;
    const bool good = hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&t, e0, e1) == hipSuccess &&
                      hipGetLastError() == hipSuccess;
    hipFree(out);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (!good || t <= 0.f) return fail(SPGM_E_DEVICE, "spgm_calibrate: timing failed");
    // chain steps per lane: 8 chains x iters (kind 3: one entry body per chain step)
    *ops_per_s = (double)grid * 256.0 * 8.0 * (double)iters / (1e-3 * (double)t);
    if (ms) *ms = (double)t;
    return ok();
}

int spgm_plan_launch_shape(const spgm_plan *p, int32_t B, int32_t *fwd_splits, int32_t *fwd_waves,
                           int32_t *adj_splits, int32_t *adj_waves) {
    if (!p) return fail(SPGM_E_INVALID, "spgm_plan_launch_shape: plan is NULL");
    if (B < 1 || B > kMaxB) return fail(SPGM_E_INVALID, "spgm_plan_launch_shape: B=%d outside [1, %d]", B, kMaxB);
    const TileShape f = fwd_shape(p, B), a = adj_shape(p, B);
    if (fwd_splits) *fwd_splits = f.splits;
    if (fwd_waves) *fwd_waves = f.waves;
    if (adj_splits) *adj_splits = a.splits;
    if (adj_waves) *adj_waves = a.waves;
    return ok();
}

// Autotuner of the ragged batch: rows per work item (the row split of every scene) among 256,
// 512, ..., 16384 (powers of two), timed on one SPGM iteration over pseudo-random rows of the given
// minibatch sizes; cached in the same file, keyed by architecture, phase mode and a hash of
// every scene's (T, R, F, grid, B).
int spgm_batch_autotune(spgm_batch *b, const int32_t *B, const char *cache_path, int32_t *rows_per_split) {
    if (!b || !B) return fail(SPGM_E_INVALID, "spgm_batch_autotune: batch and B must be non-NULL");
    const int n = (int)b->plans.size();
    for (int i = 0; i < n; ++i)
        if (B[i] < 1 || B[i] > kMaxB) return fail(SPGM_E_INVALID, "spgm_batch_autotune: scene %d: B=%d out of range", i, B[i]);
    DeviceGuard guard(b->device);
    if (hipDeviceSynchronize() != hipSuccess) return fail(SPGM_E_DEVICE, "spgm_batch_autotune: device error");
    // cache key: architecture, phase mode and every scene's (T, R, F, grid, B)
    std::ostringstream k;
    {
        hipDeviceProp_t prop;
        std::string arch = "unknown";
        if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
        uint64_t h = 1469598103934665603ull;  // FNV-1a over the scene shapes
        for (int i = 0; i < n; ++i) {
            const Geo &g = b->plans[i]->geo;
            const int v[7] = {g.T, g.R, g.F, g.nx, g.ny, g.nz, B[i]};
            for (int x : v) {
                h ^= (uint64_t)(uint32_t)x;
                h *= 1099511628211ull;
            }
        }
        k << arch << "|batch|phase" << b->phase_mode << "|n" << n << "|h" << std::hex << h;
    }
    std::string path = cache_path ? cache_path : "";
    if (path.empty() && std::getenv("SPGM_TUNE_CACHE")) path = std::getenv("SPGM_TUNE_CACHE");
    std::map<std::string, std::vector<double>> cache;
    if (!path.empty()) cache = read_cache(path);
    const auto hit = cache.find(k.str());
    if (hit != cache.end() && !hit->second.empty()) {
        const int r = (int)hit->second[0];
        b->rows_per_split = (r > 0 && r % kWave == 0) ? r : kBatchRowsPerSplit;
    } else {
        // timing inputs per scene: uniform pseudo-random rows, measurements and a zero iterate
        std::vector<int32_t *> rows(n, nullptr);
        std::vector<float2 *> ys(n, nullptr), ss(n, nullptr);
        int rc = SPGM_OK;
        uint64_t x = 0x9E3779B97F4A7C15ull;
        for (int i = 0; i < n && !rc; ++i) {
            const spgm_plan *p = b->plans[i];
            std::vector<int32_t> hr(B[i]);
            for (int j = 0; j < B[i]; ++j) {
                x ^= x << 13;
                x ^= x >> 7;
                x ^= x << 17;
                hr[j] = (int32_t)(x % (uint64_t)p->M);
            }
            if (hipMalloc(&rows[i], sizeof(int32_t) * B[i]) != hipSuccess ||
                hipMalloc(&ys[i], sizeof(float2) * (size_t)p->M) != hipSuccess ||
                hipMalloc(&ss[i], sizeof(float2) * (size_t)p->N) != hipSuccess)
                rc = fail(SPGM_E_NOMEM, "spgm_batch_autotune: allocation failed");
            else if (hipMemcpy(rows[i], hr.data(), sizeof(int32_t) * B[i], hipMemcpyHostToDevice) != hipSuccess ||
                     hipMemset(ys[i], 0, sizeof(float2) * (size_t)p->M) != hipSuccess ||
                     hipMemset(ss[i], 0, sizeof(float2) * (size_t)p->N) != hipSuccess)
                rc = fail(SPGM_E_DEVICE, "spgm_batch_autotune: copy failed");
        }
        std::vector<float> eta(n, 1.f), alpha(n, 0.f);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
            rc = fail(SPGM_E_NOMEM, "spgm_batch_autotune: event creation failed");
        const int saved_wg = b->max_wg;
        b->max_wg = 0;
        double best = 1e30;
        int best_r = kBatchRowsPerSplit;
        for (int r : {256, 512, 1024, 2048, 4096, 8192, 16384}) {
            if (rc) break;
            b->rows_per_split = r;
            float tbest = 1e30f;
            for (int rep = 0; rep < 3 && !rc; ++rep) {
                hipEventRecord(e0, nullptr);
                rc = spgm_batch_solve(b, 1, B, rows.data(), (const void *const *)ys.data(), (void *const *)ss.data(),
                                      eta.data(), alpha.data(), 0, nullptr);
                float ms = 0.f;
                if (!rc && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    rc = fail(SPGM_E_DEVICE, "spgm_batch_autotune: timing failed");
                if (!rc && rep > 0) tbest = std::min(tbest, ms);
            }
            if (!rc && tbest < best) {
                best = tbest;
                best_r = r;
            }
        }
        b->max_wg = saved_wg;
        for (int i = 0; i < n; ++i) {
            hipFree(rows[i]);
            hipFree(ys[i]);
            hipFree(ss[i]);
        }
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        if (rc) {
            b->rows_per_split = kBatchRowsPerSplit;
            return rc;
        }
        b->rows_per_split = best_r;
        if (!path.empty()) {
            cache[k.str()] = {(double)best_r, best};
            write_cache(path, cache);
        }
    }
    if (rows_per_split) *rows_per_split = b->rows_per_split;
    return ok();
}

int spgm_batch_options(spgm_batch *b, int32_t max_workgroups, int32_t rows_per_split) {
    if (!b) return fail(SPGM_E_INVALID, "spgm_batch_options: batch is NULL");
    if (max_workgroups < 0) return fail(SPGM_E_INVALID, "spgm_batch_options: max_workgroups must be >= 0");
    if (rows_per_split < 0 || (rows_per_split > 0 && rows_per_split % kWave != 0))
        return fail(SPGM_E_INVALID, "spgm_batch_options: rows_per_split must be 0 or a positive multiple of %d", kWave);
    b->max_wg = max_workgroups;
    b->rows_per_split = rows_per_split > 0 ? rows_per_split : kBatchRowsPerSplit;
    return ok();
}

int spgm_batch_status(spgm_batch *b, int32_t *status) {
    if (!b || !status) return fail(SPGM_E_INVALID, "spgm_batch_status: batch and status must be non-NULL");
    DeviceGuard guard(b->device);
    int hval = 0;
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(&hval, b->d_status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemset(b->d_status, 0, sizeof(int)) != hipSuccess)
        return fail(SPGM_E_DEVICE, "spgm_batch_status: device error");
    *status = hval ? SPGM_E_BADROW : SPGM_OK;
    return ok();
}

int spgm_plan_status(spgm_plan *p, int32_t *status) {
    if (!p || !status) return fail(SPGM_E_INVALID, "spgm_plan_status: plan and status must be non-NULL");
    DeviceGuard guard(p->device);
    int h = 0;
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(&h, p->d_status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemset(p->d_status, 0, sizeof(int)) != hipSuccess)
        return fail(SPGM_E_DEVICE, "spgm_plan_status: device error");
    *status = h ? SPGM_E_BADROW : SPGM_OK;
    return ok();
}

int spgm_plan_timing(spgm_plan *p, int32_t enable) {
    if (!p) return fail(SPGM_E_INVALID, "spgm_plan_timing: plan is NULL");
    p->timing = enable != 0;
    return ok();
}

int spgm_plan_timing_read(spgm_plan *p, double *fwd_ms, int64_t *fwd_n, double *adj_ms, int64_t *adj_n) {
    if (!p) return fail(SPGM_E_INVALID, "spgm_plan_timing_read: plan is NULL");
    DeviceGuard guard(p->device);
    if (hipDeviceSynchronize() != hipSuccess) return fail(SPGM_E_DEVICE, "spgm_plan_timing_read: device error");
    auto total = [](const std::vector<hipEvent_t> &pool, size_t used) {
        double ms = 0.0;
        for (size_t k = 0; k < used; ++k) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, pool[2 * k], pool[2 * k + 1]) == hipSuccess) ms += t;
        }
        return ms;
    };
    if (fwd_ms) *fwd_ms = total(p->ev_fwd, p->n_fwd);
    if (adj_ms) *adj_ms = total(p->ev_adj, p->n_adj);
    if (fwd_n) *fwd_n = (int64_t)p->n_fwd;
    if (adj_n) *adj_n = (int64_t)p->n_adj;
    p->n_fwd = p->n_adj = 0;
    return ok();
}

int spgm_forward_batched(spgm_plan *p, const int32_t *rows, int32_t B, int32_t K, const void *S, void *Y,
                         int32_t prec, void *stream) {
    int rc;
    if ((rc = mm_check(p, rows, B, K, prec, "spgm_forward_batched"))) return rc;
    if (!S || !Y) return fail(SPGM_E_INVALID, "spgm_forward_batched: S and Y must be non-NULL");
    DeviceGuard guard(p->device);
    if ((rc = ensure_mm(p, B))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = run_sort(p, rows, B, 1, p->d_srt, st))) return rc;
    rc = prec == SPGM_MM_FP16
             ? mm_forward<SPGM_MM_FP16>(p, p->d_srt, rows, B, K, (const float2 *)S, (float2 *)Y, st)
             : mm_forward<SPGM_MM_BF16>(p, p->d_srt, rows, B, K, (const float2 *)S, (float2 *)Y, st);
    return rc ? rc : ok();
}

int spgm_adjoint_batched(spgm_plan *p, const int32_t *rows, int32_t B, int32_t K, const void *R, void *G,
                         int32_t prec, void *stream) {
    int rc;
    if ((rc = mm_check(p, rows, B, K, prec, "spgm_adjoint_batched"))) return rc;
    if (!R || !G) return fail(SPGM_E_INVALID, "spgm_adjoint_batched: R and G must be non-NULL");
    DeviceGuard guard(p->device);
    if ((rc = ensure_mm(p, B))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = run_sort(p, rows, B, 1, p->d_srt, st))) return rc;
    rc = prec == SPGM_MM_FP16 ? mm_adjoint<SPGM_MM_FP16>(p, p->d_srt, B, K, (const float2 *)R, (float2 *)G, st)
                              : mm_adjoint<SPGM_MM_BF16>(p, p->d_srt, B, K, (const float2 *)R, (float2 *)G, st);
    return rc ? rc : ok();
}

int spgm_step_batched(spgm_plan *p, const int32_t *rows, int32_t B, int32_t K, const void *Ym, void *S, float eta,
                      float alpha, int32_t prec, void *stream) {
    int rc;
    if ((rc = mm_check(p, rows, B, K, prec, "spgm_step_batched"))) return rc;
    if ((rc = check_step_args(Ym, S, eta, alpha))) return rc;
    DeviceGuard guard(p->device);
    if ((rc = ensure_mm(p, B))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = run_sort(p, rows, B, 1, p->d_srt, st))) return rc;
    if ((rc = mm_step_any(p, prec, p->d_srt, rows, B, K, (const float2 *)Ym, (float2 *)S, eta, alpha, st))) return rc;
    return ok();
}

int spgm_solve_batched(spgm_plan *p, const int32_t *rows, int32_t iters, int32_t B, int32_t K, const void *Ym,
                       void *S, float eta, float alpha, int32_t prec, void *stream) {
    int rc;
    if ((rc = mm_check(p, rows, B, K, prec, "spgm_solve_batched"))) return rc;
    if ((rc = check_step_args(Ym, S, eta, alpha))) return rc;
    if (iters < 0) return fail(SPGM_E_INVALID, "spgm_solve_batched: iters must be >= 0");
    if (iters == 0) return ok();
    DeviceGuard guard(p->device);
    if ((rc = ensure_mm(p, B))) return rc;
    const int per = (int)std::max<size_t>(1, std::min<size_t>((size_t)iters, kSolveSortRows / (size_t)B));
    if ((rc = ensure_sorted_batch(p, (size_t)per * B))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const bool chain = mm_chain_ok(p, B, K);
    bool packed = false;  // the packed operand holds the current S
    for (int i0 = 0; i0 < iters; i0 += per) {
        const int cnt = std::min(per, iters - i0);
        const int32_t *ri = rows + (size_t)i0 * B;
        if ((rc = run_sort(p, ri, B, cnt, p->d_srt_all, st))) return rc;
        for (int i = 0; i < cnt; ++i) {
            const bool s2_out = chain && i0 + i + 1 < iters;
            if ((rc = mm_step_any(p, prec, p->d_srt_all + (size_t)i * B, ri + (size_t)i * B, B, K, (const float2 *)Ym,
                                  (float2 *)S, eta, alpha, st, packed, s2_out)))
                return rc;
            packed = s2_out;
        }
    }
    return ok();
}

int spgm_forward_structured(spgm_plan *p, const int32_t *f_idx, int32_t nf, const int32_t *t_idx, int32_t nt,
                            const int32_t *r_idx, int32_t nr, const void *s, void *y, void *stream) {
    const SFArgs a{f_idx, t_idx, r_idx, nf, nt, nr, nf * nt * nr};
    int rc;
    if ((rc = sf_check(p, a, "spgm_forward_structured"))) return rc;
    if (!s || !y) return fail(SPGM_E_INVALID, "spgm_forward_structured: s and y must be non-NULL");
    DeviceGuard guard(p->device);
    hipStream_t st = (hipStream_t)stream;
    if ((rc = sf_prepare(p, a, st))) return rc;
    if ((rc = sf_forward_partials(p, a, (const float2 *)s, st))) return rc;
    if ((rc = run_row_reduce(p, p->d_srt, p->d_sf_rows, a.B, nullptr, (float2 *)y, nullptr, st))) return rc;
    return ok();
}

int spgm_adjoint_structured(spgm_plan *p, const int32_t *f_idx, int32_t nf, const int32_t *t_idx, int32_t nt,
                            const int32_t *r_idx, int32_t nr, const void *r, void *g, void *stream) {
    const SFArgs a{f_idx, t_idx, r_idx, nf, nt, nr, nf * nt * nr};
    int rc;
    if ((rc = sf_check(p, a, "spgm_adjoint_structured"))) return rc;
    if (!r || !g) return fail(SPGM_E_INVALID, "spgm_adjoint_structured: r and g must be non-NULL");
    DeviceGuard guard(p->device);
    hipStream_t st = (hipStream_t)stream;
    if ((rc = sf_prepare(p, a, st))) return rc;
    k_gather_scale<<<(a.B + 255) / 256, 256, 0, st>>>(p->geo, p->d_srt, a.B, (const float2 *)r, p->d_rs);
    if ((rc = launch_check("gather"))) return rc;
    if ((rc = sf_adjoint_partials(p, a, st))) return rc;
    k_col_reduce<<<(int)((p->N + 255) / 256), 256, 0, st>>>(p->d_gpart, 1, (int)p->N, (float2 *)g, nullptr, 0.f, 0.f);
    if ((rc = launch_check("column reduce"))) return rc;
    return ok();
}

int spgm_step_structured(spgm_plan *p, const int32_t *f_idx, int32_t nf, const int32_t *t_idx, int32_t nt,
                         const int32_t *r_idx, int32_t nr, const void *y, void *s, float eta, float alpha,
                         void *stream) {
    const SFArgs a{f_idx, t_idx, r_idx, nf, nt, nr, nf * nt * nr};
    int rc;
    if ((rc = sf_check(p, a, "spgm_step_structured"))) return rc;
    if ((rc = check_step_args(y, s, eta, alpha))) return rc;
    DeviceGuard guard(p->device);
    if ((rc = sf_step(p, a, (const float2 *)y, (float2 *)s, eta, alpha, (hipStream_t)stream))) return rc;
    return ok();
}

int spgm_solve_structured(spgm_plan *p, const int32_t *f_idx, int32_t nf, const int32_t *t_idx, int32_t nt,
                          const int32_t *r_idx, int32_t nr, int32_t iters, const void *y, void *s, float eta,
                          float alpha, void *stream) {
    const SFArgs a0{f_idx, t_idx, r_idx, nf, nt, nr, nf * nt * nr};
    int rc;
    if ((rc = sf_check(p, a0, "spgm_solve_structured"))) return rc;
    if ((rc = check_step_args(y, s, eta, alpha))) return rc;
    if (iters < 0) return fail(SPGM_E_INVALID, "spgm_solve_structured: iters must be >= 0");
    DeviceGuard guard(p->device);
    for (int k = 0; k < iters; ++k) {
        const SFArgs a{f_idx + (size_t)k * nf, t_idx + (size_t)k * nt, r_idx + (size_t)k * nr, nf, nt, nr, a0.B};
        if ((rc = sf_step(p, a, (const float2 *)y, (float2 *)s, eta, alpha, (hipStream_t)stream))) return rc;
    }
    return ok();
}

}  // extern "C"
