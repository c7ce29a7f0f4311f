// mech.hip -- gfx950 kernels and C-ABI runtime of the agent-mechanics step (libmech.so).
//
// One step, all on the device, on the population's stream:
//   k_bin          a1+a2  voxel of every cell (FP64 key) and an integer-atomic histogram
//   k_scan_reduce  a3     per-tile sums of (count, occupied) packed in 64 bits
//   k_scan_top            exclusive scan of the tile sums (one workgroup)
//   k_scan_down           voxel_start (exclusive prefix), occupied-voxel list, count reset
//   k_scatter      a4     cells into their voxel's segment (arbitrary order inside it)
//   k_rank_gather  a4+a5  rank inside the segment by ascending id -> final slot; gather of
//                         the cell state into voxel order (+ the float shadow)
//   k_force_*      a6+a7  27-voxel neighbour forces -> velocity, Adams-Bashforth, walls
// The paper measures the mechanics "update velocity" loop as the region that degrades
// when cells sit in memory in creation order rather than next to their neighbours in
// space (Section 5.4); here every step re-sorts cells by voxel, so the force kernel
// always reads neighbours that are contiguous in memory, and it visits only occupied
// voxels' cells (Section 5.4: skip empty voxels).
//
// State layout (structure of arrays, one entry per cell):
//   X[3]    f64  positions in the order of the last sort (integration output, binning input)
//   XS[3]   f64  positions gathered into this step's voxel order (force input)
//   R[2]    f64  radius, T[2] i32 type, ID[2] u32 cell id, VP[2][3] v_prev (f64 or f32):
//                double-buffered; parity p holds them in the order of X
//   SH      float4 (x, y, z, r) in voxel order, FP32 variants only
// Binning scratch: vid_cur, off, tmp_key, tmp_src, vid_sorted (u32 per cell);
// count, voxel_start, occ (u32 per voxel); tile sums (u64 per 2048 voxels).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "mech.h"

namespace {

// ------------------------------------------------------------------------ errors

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[768];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(MECH_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

// ------------------------------------------------------------------------ constants

constexpr int BLOCK = 256;                 // threads per workgroup (4 wave64)
constexpr int WAVE = 64;
constexpr int SCAN_PER_THREAD = 8;
constexpr int SCAN_TILE = BLOCK * SCAN_PER_THREAD;
constexpr uint32_t N_XCD = 8;              // MI355X: 8 accelerator complex dies

// ------------------------------------------------------------------------ kernel args

struct GridArgs {
    double lo[3];
    double inv_h;
    int32_t n[3];
    uint32_t V;
};

struct PhysArgs {
    double lo[3], hi[3];
    double dt, c_rep, alpha, c_adh0;
    double r_max;              // largest radius of the population
    float c_rep_f, alpha_f, c_adh0_f, r_max_f;
    int32_t n_types;
    int32_t nx, ny, nz;
};

// Workgroups are dealt to the 8 XCDs round robin; renumber them so that each XCD gets a
// contiguous run of the voxel-ordered cells and its own L2 keeps the shared neighbours.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb)
{
    uint32_t xcd = b % N_XCD, k = b / N_XCD, q = nb / N_XCD, r = nb % N_XCD;
    return xcd < r ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

// a1: voxel of a position.  (x - lo) * (1/h) is a subtraction then a product, so no
// fused form exists and the result is the IEEE value of the written expression.
__device__ __forceinline__ uint32_t voxel_key(double x, double y, double z, const GridArgs& g)
{
    double f0 = floor((x - g.lo[0]) * g.inv_h);
    double f1 = floor((y - g.lo[1]) * g.inv_h);
    double f2 = floor((z - g.lo[2]) * g.inv_h);
    f0 = fmin(fmax(f0, 0.0), (double)(g.n[0] - 1));
    f1 = fmin(fmax(f1, 0.0), (double)(g.n[1] - 1));
    f2 = fmin(fmax(f2, 0.0), (double)(g.n[2] - 1));
    uint32_t k0 = (uint32_t)f0, k1 = (uint32_t)f1, k2 = (uint32_t)f2;
    return k0 + (uint32_t)g.n[0] * (k1 + (uint32_t)g.n[1] * k2);
}

// ------------------------------------------------------------------------ wave / block helpers

template <typename T>
__device__ __forceinline__ T wave_sum(T x)
{
    for (int o = WAVE / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, WAVE);
    return x;
}

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t x)
{
    const int lane = threadIdx.x & (WAVE - 1);
    for (int o = 1; o < WAVE; o <<= 1) {
        uint64_t y = __shfl_up(x, o, WAVE);
        if (lane >= o) x += y;
    }
    return x;
}

// Exclusive scan over the workgroup; *total receives the workgroup sum.
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t x, uint64_t* sh, uint64_t* total)
{
    uint64_t inc = wave_incl_scan(x);
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    if (lane == WAVE - 1) sh[w] = inc;
    __syncthreads();
    uint64_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < BLOCK / WAVE; ++i) {
        if (i < w) off += sh[i];
        tot += sh[i];
    }
    __syncthreads();
    *total = tot;
    return off + inc - x;
}

// ------------------------------------------------------------------------ a1 + a2

__global__ __launch_bounds__(BLOCK) void k_bin(const double* __restrict__ px,
                                               const double* __restrict__ py,
                                               const double* __restrict__ pz, uint32_t n,
                                               GridArgs g, uint32_t* __restrict__ count,
                                               uint32_t* __restrict__ vid,
                                               uint32_t* __restrict__ off)
{
    uint32_t s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= n) return;
    uint32_t v = voxel_key(px[s], py[s], pz[s], g);
    off[s] = atomicAdd(&count[v], 1u);
    vid[s] = v;
}

// ------------------------------------------------------------------------ a3

// Low 32 bits: cells; high 32 bits: occupied voxels.  Both sums stay below 2^32.
__device__ __forceinline__ uint64_t pack_count(uint32_t c)
{
    return (uint64_t)c | ((uint64_t)(c != 0u) << 32);
}

__global__ __launch_bounds__(BLOCK) void k_scan_reduce(const uint32_t* __restrict__ count,
                                                       uint32_t V, uint64_t* __restrict__ tsum)
{
    __shared__ uint64_t sh[BLOCK / WAVE];
    const uint32_t base = blockIdx.x * SCAN_TILE;
    uint64_t acc = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        uint32_t v = base + k * BLOCK + threadIdx.x;
        if (v < V) acc += pack_count(count[v]);
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int i = 0; i < BLOCK / WAVE; ++i) t += sh[i];
        tsum[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(BLOCK) void k_scan_top(uint64_t* __restrict__ tsum, uint32_t nt,
                                                    uint32_t* __restrict__ voxel_start,
                                                    uint32_t V, uint32_t* __restrict__ n_occ)
{
    __shared__ uint64_t sh[BLOCK / WAVE];
    uint64_t carry = 0;
    for (uint32_t base = 0; base < nt; base += BLOCK) {
        uint32_t i = base + threadIdx.x;
        uint64_t x = i < nt ? tsum[i] : 0;
        uint64_t tot;
        uint64_t ex = block_excl_scan(x, sh, &tot);
        if (i < nt) tsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        voxel_start[V] = (uint32_t)carry;
        *n_occ = (uint32_t)(carry >> 32);
    }
}

__global__ __launch_bounds__(BLOCK) void k_scan_down(uint32_t* __restrict__ count, uint32_t V,
                                                     const uint64_t* __restrict__ toff,
                                                     uint32_t* __restrict__ voxel_start,
                                                     uint32_t* __restrict__ occ)
{
    __shared__ uint32_t tile[SCAN_TILE];
    __shared__ uint64_t sh[BLOCK / WAVE];
    const uint32_t base = blockIdx.x * SCAN_TILE;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        uint32_t v = base + k * BLOCK + threadIdx.x;
        tile[k * BLOCK + threadIdx.x] = v < V ? count[v] : 0u;
    }
    __syncthreads();
    uint64_t loc[SCAN_PER_THREAD];
    uint64_t sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        loc[k] = sum;
        sum += pack_count(tile[threadIdx.x * SCAN_PER_THREAD + k]);
    }
    uint64_t tot;
    uint64_t off = toff[blockIdx.x] + block_excl_scan(sum, sh, &tot);
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        uint32_t v = base + threadIdx.x * SCAN_PER_THREAD + k;
        if (v < V) {
            uint64_t e = off + loc[k];
            voxel_start[v] = (uint32_t)e;
            if (tile[threadIdx.x * SCAN_PER_THREAD + k]) occ[(uint32_t)(e >> 32)] = v;
        }
    }
    // the histogram of the next step starts from zero
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        uint32_t v = base + k * BLOCK + threadIdx.x;
        if (v < V) count[v] = 0u;
    }
}

// ------------------------------------------------------------------------ a4 + a5

__global__ __launch_bounds__(BLOCK) void k_scatter(uint32_t n, const uint32_t* __restrict__ vid,
                                                   const uint32_t* __restrict__ off,
                                                   const uint32_t* __restrict__ voxel_start,
                                                   const uint32_t* __restrict__ id_cur,
                                                   uint32_t* __restrict__ tmp_key,
                                                   uint32_t* __restrict__ tmp_src)
{
    uint32_t s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= n) return;
    uint32_t p = voxel_start[vid[s]] + off[s];
    tmp_key[p] = id_cur[s];
    tmp_src[p] = s;
}

template <typename VPT>
struct GatherArgs {
    const double* X[3];
    double* XS[3];
    const double* R_cur;
    double* R_new;
    const int32_t* T_cur;
    int32_t* T_new;
    uint32_t* ID_new;
    const VPT* VP_cur[3];
    VPT* VP_new[3];
    float4* SH;              // nullptr in FP64
    const uint32_t* vid_cur;
    const uint32_t* tmp_key;
    const uint32_t* tmp_src;
    const uint32_t* voxel_start;
    uint32_t* vid_sorted;
};

// Segments are short (tens of cells), so each cell counts the smaller ids of its own
// segment directly; the cost is below that of the force loop over the same cells.
template <typename VPT>
__global__ __launch_bounds__(BLOCK) void k_rank_gather(uint32_t n, GatherArgs<VPT> a)
{
    uint32_t p = blockIdx.x * BLOCK + threadIdx.x;
    if (p >= n) return;
    const uint32_t s = a.tmp_src[p];
    const uint32_t key = a.tmp_key[p];
    const uint32_t v = a.vid_cur[s];
    const uint32_t b = a.voxel_start[v], e = a.voxel_start[v + 1];
    uint32_t rank = 0;
    for (uint32_t q = b; q < e; ++q) rank += a.tmp_key[q] < key;
    const uint32_t d = b + rank;
    double x = a.X[0][s], y = a.X[1][s], z = a.X[2][s];
    double r = a.R_cur[s];
    a.XS[0][d] = x;
    a.XS[1][d] = y;
    a.XS[2][d] = z;
    a.R_new[d] = r;
    a.T_new[d] = a.T_cur[s];
    a.ID_new[d] = key;
#pragma unroll
    for (int c = 0; c < 3; ++c) a.VP_new[c][d] = a.VP_cur[c][s];
    a.vid_sorted[d] = v;
    if (a.SH) a.SH[d] = make_float4((float)x, (float)y, (float)z, (float)r);
}

__global__ __launch_bounds__(BLOCK) void k_copy_positions(uint32_t n, const double* __restrict__ a0,
                                                          const double* __restrict__ a1,
                                                          const double* __restrict__ a2,
                                                          double* __restrict__ b0,
                                                          double* __restrict__ b1,
                                                          double* __restrict__ b2)
{
    uint32_t s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= n) return;
    b0[s] = a0[s];
    b1[s] = a1[s];
    b2[s] = a2[s];
}

// ------------------------------------------------------------------------ a6 + a7

__device__ __forceinline__ double reflect(double x, double lo, double hi)
{
    if (x < lo) x = 2.0 * lo - x;
    if (x > hi) x = 2.0 * hi - x;
    return fmin(fmax(x, lo), hi);
}

template <typename VPT>
struct ForceArgs {
    const double* XS[3];
    const double* R;
    const int32_t* T;
    const float4* SH;
    const uint32_t* vid_sorted;
    const uint32_t* voxel_start;
    const double* cadh;        // n_types^2 (FP64)
    const float* cadh_f;       // n_types^2 (FP32)
    VPT* VP[3];                // read v_prev, write v (in place, own element)
    double* X[3];              // new positions
    unsigned long long* stats; // [0] interactions, [1] candidates
    int euler;
};

// FP64 pair term.  d2 and the in-range test are evaluated without contraction so the
// decision is the exact IEEE result of d2 = dx*dx + dy*dy + dz*dz < (alpha (ri+rj))^2.
__device__ __forceinline__ bool pair64(double xi, double yi, double zi, double ri, double xj,
                                       double yj, double zj, double rj, double alpha,
                                       double c_rep, double cadh, double& ax, double& ay,
                                       double& az)
{
    double dx, dy, dz, d2, R, RA;
    {
#pragma clang fp contract(off)
        dx = xi - xj;
        dy = yi - yj;
        dz = zi - zj;
        d2 = dx * dx + dy * dy + dz * dz;
        R = ri + rj;
        RA = alpha * R;
        if (!(d2 > 0.0 && d2 < RA * RA)) return false;
    }
    double d = sqrt(d2);
    double w = 0.0;
    if (d < R) {
        double u = 1.0 - d / R;
        w = c_rep * u * u;
    }
    double a = 1.0 - d / RA;
    w -= cadh * a * a;
    double s = w / d;
    ax += s * dx;
    ay += s * dy;
    az += s * dz;
    return true;
}

// FP32 pair term on the float shadow: same decision as the float oracle
// (d2 by two fused multiply-adds, R and R_A rounded to float).
template <bool KAHAN>
__device__ __forceinline__ bool pair32(float xi, float yi, float zi, float ri, float4 q,
                                       float alpha, float c_rep, float cadh, float* acc,
                                       float* cmp)
{
    float dx, dy, dz, d2, R, RA;
    {
#pragma clang fp contract(off)
        dx = xi - q.x;
        dy = yi - q.y;
        dz = zi - q.z;
        d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
        R = ri + q.w;
        RA = alpha * R;
        if (!(d2 > 0.0f && d2 < RA * RA)) return false;
    }
    float inv_d = __builtin_amdgcn_rsqf(d2);
    float d = d2 * inv_d;
    float w = 0.0f;
    if (d < R) {
        float u = 1.0f - d * __builtin_amdgcn_rcpf(R);
        w = c_rep * u * u;
    }
    float a = 1.0f - d * __builtin_amdgcn_rcpf(RA);
    w -= cadh * a * a;
    float s = w * inv_d;
    float t[3] = {s * dx, s * dy, s * dz};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (KAHAN) {
            float y = t[c] - cmp[c];
            float tt = acc[c] + y;
            cmp[c] = (tt - acc[c]) - y;
            acc[c] = tt;
        } else {
            acc[c] += t[c];
        }
    }
    return true;
}

// Running counters are spread over STAT_SLOTS pairs (summed when read): device-scope
// atomics on one address from every wave of the GPU serialise at the memory side.
constexpr uint32_t STAT_SLOTS = 1024;

__device__ __forceinline__ void add_stats(unsigned long long* stats, uint32_t inter, uint32_t cand)
{
    unsigned long long a = wave_sum<unsigned long long>(inter);
    unsigned long long b = wave_sum<unsigned long long>(cand);
    if ((threadIdx.x & (WAVE - 1)) == 0 && (a | b)) {
        const uint32_t slot = (blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE) % STAT_SLOTS;
        atomicAdd(&stats[2 * slot], a);
        atomicAdd(&stats[2 * slot + 1], b);
    }
}

// One thread per cell in voxel order.  The 27 neighbour voxels are visited as 9 rows
// (dz, dy); the three voxels of a row (dx = -1, 0, 1) are adjacent in voxel order, so a
// row is one contiguous range of the sorted arrays, read in the oracle's order.
// PREC: 0 FP64, 1 FP32, 2 FP32 + Kahan.  MULTI: more than one cell type.
template <int PREC, bool MULTI, typename VPT>
__global__ __launch_bounds__(BLOCK) void k_force_rows(uint32_t n, PhysArgs P, ForceArgs<VPT> a)
{
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t i = blk * BLOCK + threadIdx.x;
    uint32_t inter = 0, cand = 0;
    if (i < n) {
        const uint32_t vox = a.vid_sorted[i];
        const int kx = (int)(vox % (uint32_t)P.nx);
        const int ky = (int)((vox / (uint32_t)P.nx) % (uint32_t)P.ny);
        const int kz = (int)(vox / ((uint32_t)P.nx * (uint32_t)P.ny));
        const int x0 = kx > 0 ? kx - 1 : 0;
        const int x1 = kx < P.nx - 1 ? kx + 1 : P.nx - 1;
        const int ti = MULTI ? a.T[i] : 0;
        const double xi = a.XS[0][i], yi = a.XS[1][i], zi = a.XS[2][i];
        double vx, vy, vz;
        if (PREC == 0) {
            const double ri = a.R[i];
            double ax = 0.0, ay = 0.0, az = 0.0;
            for (int dz = -1; dz <= 1; ++dz) {
                const int z = kz + dz;
                if (z < 0 || z >= P.nz) continue;
                for (int dy = -1; dy <= 1; ++dy) {
                    const int y = ky + dy;
                    if (y < 0 || y >= P.ny) continue;
                    const uint32_t row = (uint32_t)P.nx * ((uint32_t)y + (uint32_t)P.ny * (uint32_t)z);
                    const uint32_t b = a.voxel_start[row + x0], e = a.voxel_start[row + x1 + 1];
                    cand += e - b;
                    for (uint32_t j = b; j < e; ++j) {
                        const double c = MULTI ? a.cadh[ti * P.n_types + a.T[j]] : P.c_adh0;
                        inter += pair64(xi, yi, zi, ri, a.XS[0][j], a.XS[1][j], a.XS[2][j],
                                        a.R[j], P.alpha, P.c_rep, c, ax, ay, az);
                    }
                }
            }
            vx = ax;
            vy = ay;
            vz = az;
        } else {
            const float4 me = a.SH[i];
            float acc[3] = {0.f, 0.f, 0.f}, cmp[3] = {0.f, 0.f, 0.f};
            for (int dz = -1; dz <= 1; ++dz) {
                const int z = kz + dz;
                if (z < 0 || z >= P.nz) continue;
                for (int dy = -1; dy <= 1; ++dy) {
                    const int y = ky + dy;
                    if (y < 0 || y >= P.ny) continue;
                    const uint32_t row = (uint32_t)P.nx * ((uint32_t)y + (uint32_t)P.ny * (uint32_t)z);
                    const uint32_t b = a.voxel_start[row + x0], e = a.voxel_start[row + x1 + 1];
                    cand += e - b;
                    for (uint32_t j = b; j < e; ++j) {
                        const float c = MULTI ? a.cadh_f[ti * P.n_types + a.T[j]] : P.c_adh0_f;
                        inter += pair32<PREC == 2>(me.x, me.y, me.z, me.w, a.SH[j], P.alpha_f,
                                                   P.c_rep_f, c, acc, cmp);
                    }
                }
            }
            vx = acc[0];
            vy = acc[1];
            vz = acc[2];
        }
        cand -= 1;  // the cell itself
        // a7: two-step Adams-Bashforth, reflecting walls, history
        const double v[3] = {vx, vy, vz};
        const double x[3] = {xi, yi, zi};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double vp = a.euler ? v[c] : (double)a.VP[c][i];
            const double xn = x[c] + P.dt * (1.5 * v[c] - 0.5 * vp);
            a.X[c][i] = reflect(xn, P.lo[c], P.hi[c]);
            a.VP[c][i] = (VPT)v[c];
        }
    }
    add_stats(a.stats, inter, cand);
}

// ------------------------------------------------------------------------ a6 + a7, per-cell lists

// In-range decision only (the term is computed later from a list); the same
// expressions, uncontracted, as in pair64 / pair32.
__device__ __forceinline__ bool in_range64(const double4& me, const double4& c, double alpha)
{
#pragma clang fp contract(off)
    const double dx = me.x - c.x, dy = me.y - c.y, dz = me.z - c.z;
    const double d2 = dx * dx + dy * dy + dz * dz;
    const double RA = alpha * (me.w + c.w);
    return d2 > 0.0 && d2 < RA * RA;
}

__device__ __forceinline__ bool in_range32(const float4& me, const float4& c, float alpha)
{
#pragma clang fp contract(off)
    const float dx = me.x - c.x, dy = me.y - c.y, dz = me.z - c.z;
    const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
    const float RA = alpha * (me.w + c.w);
    return d2 > 0.0f && d2 < RA * RA;
}

constexpr int FC_LIST = 16;    // listed candidates a lane holds before a flush
constexpr int FC_UNROLL = 4;   // candidates tested per loop trip (independent loads in flight)

// One thread per cell in voxel order.  Each lane walks its 9 neighbour rows (dz, dy;
// the three voxels of a row are adjacent in voxel order) and only prefilters the
// candidates, four loads in flight per trip: a candidate is listed in LDS when
//   d2 < (alpha (r_i + r_max))^2,
// which every interacting pair satisfies (r_j <= r_max and rounding is monotonic; d2
// is the same expression as in the exact test).  When a list fills, and at the end,
// the lanes evaluate their listed candidates together with the exact decision and
// pair term of pair64 / pair32, in candidate order, so each sum is still taken in the
// fixed neighbour order and the rare interacting pairs do not make the wave diverge.
// Lanes of one voxel read the same candidate at the same time (one cache line).
template <int PREC, bool MULTI, typename VPT>
__global__ __launch_bounds__(BLOCK) void k_force_cells(uint32_t n, PhysArgs P, ForceArgs<VPT> a)
{
    using Real = typename std::conditional<PREC == 0, double, float>::type;
    __shared__ uint32_t s_list[BLOCK / WAVE][FC_LIST][WAVE];

    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    const uint32_t i = xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    const bool valid = i < n;
    const uint32_t ii = valid ? i : n - 1;  // n >= 1: idle lanes mirror the last cell
    const uint32_t vox = a.vid_sorted[ii];
    const int kx = (int)(vox % (uint32_t)P.nx);
    const int ky = (int)((vox / (uint32_t)P.nx) % (uint32_t)P.ny);
    const int kz = (int)(vox / ((uint32_t)P.nx * (uint32_t)P.ny));
    const int x0 = kx > 0 ? kx - 1 : 0;
    const int x1 = kx < P.nx - 1 ? kx + 1 : P.nx - 1;
    Real xi, yi, zi, ri;
    if constexpr (PREC == 0) {
        xi = a.XS[0][ii];
        yi = a.XS[1][ii];
        zi = a.XS[2][ii];
        ri = a.R[ii];
    } else {
        const float4 m = a.SH[ii];
        xi = m.x;
        yi = m.y;
        zi = m.z;
        ri = m.w;
    }
    Real T;
    {
#pragma clang fp contract(off)
        const Real reach = (PREC == 0 ? (Real)P.alpha : (Real)P.alpha_f) *
                           (ri + (PREC == 0 ? (Real)P.r_max : (Real)P.r_max_f));
        T = reach * reach;
    }
    const int ti = MULTI ? a.T[ii] : 0;
    Real acc[3] = {0, 0, 0}, cmp[3] = {0, 0, 0};
    uint32_t inter = 0, cand = 0;
    uint32_t* const list0 = &s_list[w][0][lane];
    uint32_t* const list_hi = list0 + (FC_LIST - FC_UNROLL) * WAVE;
    uint32_t* lp = list0;

    auto near = [&](Real cx, Real cy, Real cz) -> bool {
#pragma clang fp contract(off)
        const Real dx = xi - cx, dy = yi - cy, dz = zi - cz;
        Real d2;
        if constexpr (PREC == 0)
            d2 = dx * dx + dy * dy + dz * dz;
        else
            d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
        return d2 < T;
    };
    auto flush = [&]() {
        const uint32_t cnt = (uint32_t)(lp - list0) / WAVE;
        for (uint32_t q = 0; q < (uint32_t)FC_LIST; ++q) {
            if (!__any(q < cnt)) break;
            if (q < cnt) {
                const uint32_t j = list0[q * WAVE];
                if constexpr (PREC == 0) {
                    const double cadh = MULTI ? a.cadh[ti * P.n_types + a.T[j]] : P.c_adh0;
                    inter += pair64(xi, yi, zi, ri, a.XS[0][j], a.XS[1][j], a.XS[2][j], a.R[j],
                                    P.alpha, P.c_rep, cadh, acc[0], acc[1], acc[2]);
                } else {
                    const float cadh = MULTI ? a.cadh_f[ti * P.n_types + a.T[j]] : P.c_adh0_f;
                    inter += pair32<PREC == 2>(xi, yi, zi, ri, a.SH[j], P.alpha_f, P.c_rep_f, cadh,
                                               acc, cmp);
                }
            }
        }
        lp = list0;
    };

    for (int q = 0; q < 9; ++q) {
        const int y = ky + (q % 3) - 1, z = kz + (q / 3) - 1;
        if (!valid || y < 0 || y >= P.ny || z < 0 || z >= P.nz) continue;
        const uint32_t row = (uint32_t)P.nx * ((uint32_t)y + (uint32_t)P.ny * (uint32_t)z);
        uint32_t j = a.voxel_start[row + x0];
        const uint32_t e = a.voxel_start[row + x1 + 1];
        cand += e - j;
        if constexpr (PREC == 0) {
            const double* px = a.XS[0] + j;
            const double* py = a.XS[1] + j;
            const double* pz = a.XS[2] + j;
            for (; j + FC_UNROLL <= e; j += FC_UNROLL, px += FC_UNROLL, py += FC_UNROLL, pz += FC_UNROLL) {
                double cx[FC_UNROLL], cy[FC_UNROLL], cz[FC_UNROLL];
#pragma unroll
                for (int u = 0; u < FC_UNROLL; ++u) {
                    cx[u] = px[u];
                    cy[u] = py[u];
                    cz[u] = pz[u];
                }
#pragma unroll
                for (int u = 0; u < FC_UNROLL; ++u)
                    if (near(cx[u], cy[u], cz[u])) {
                        *lp = j + u;
                        lp += WAVE;
                    }
                if (__any(lp > list_hi)) flush();
            }
            for (; j < e; ++j, ++px, ++py, ++pz) {
                if (near(*px, *py, *pz)) {
                    *lp = j;
                    lp += WAVE;
                }
                if (__any(lp > list_hi)) flush();
            }
        } else {
            const float4* sp = a.SH + j;
            for (; j + FC_UNROLL <= e; j += FC_UNROLL, sp += FC_UNROLL) {
                float4 c[FC_UNROLL];
#pragma unroll
                for (int u = 0; u < FC_UNROLL; ++u) c[u] = sp[u];
#pragma unroll
                for (int u = 0; u < FC_UNROLL; ++u)
                    if (near(c[u].x, c[u].y, c[u].z)) {
                        *lp = j + u;
                        lp += WAVE;
                    }
                if (__any(lp > list_hi)) flush();
            }
            for (; j < e; ++j, ++sp) {
                const float4 c = *sp;
                if (near(c.x, c.y, c.z)) {
                    *lp = j;
                    lp += WAVE;
                }
                if (__any(lp > list_hi)) flush();
            }
        }
    }
    flush();
    if (valid) {
        cand -= 1;  // the cell itself
        const double xs[3] = {a.XS[0][i], a.XS[1][i], a.XS[2][i]};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = (double)(acc[c] - cmp[c]);
            const double vp = a.euler ? v : (double)a.VP[c][i];
            const double xn = xs[c] + P.dt * (1.5 * v - 0.5 * vp);
            a.X[c][i] = reflect(xn, P.lo[c], P.hi[c]);
            a.VP[c][i] = (VPT)v;
        }
    }
    add_stats(a.stats, inter, cand);
}

// ------------------------------------------------------------------------ a6 + a7, LDS-staged

// Per-wave LDS: the candidates of one chunk of the 27-voxel neighbourhood (x, y, z, r),
// their types, and per-lane lists of in-range candidate indices.
constexpr int FL_WAVES = 4;                // waves per workgroup
constexpr int FL_LIST = 16;                // list entries per lane before a flush

template <int PREC> struct Stage;
template <> struct Stage<0> { using T = double4; static constexpr int CAP = 256; };
template <> struct Stage<1> { using T = float4; static constexpr int CAP = 512; };
template <> struct Stage<2> { using T = float4; static constexpr int CAP = 512; };

// Orders this wave's LDS accesses: writes by one lane are seen by the others after it.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave per occupied voxel: the waves of the grid walk the non-empty voxel list with
// a fixed stride (empty voxels cost nothing).  The wave stages its 27-voxel neighbourhood in LDS
// (9 rows, each a contiguous range of the voxel-ordered arrays) and splits its lanes
// as (target, slice): target t of r = min(64, remaining) takes lanes t, t + r, ...,
// so all 64 lanes test candidates.  A lane appends the in-range candidates of its slice
// to an LDS list and evaluates them in a batch, so the force arithmetic does not
// diverge on the rare in-range branch.  Slices are combined in a fixed order: results
// are bitwise reproducible.
template <int PREC, bool MULTI, typename VPT>
__global__ __launch_bounds__(FL_WAVES * WAVE) void k_force_lds(PhysArgs P, ForceArgs<VPT> a,
                                                               const uint32_t* __restrict__ occ,
                                                               const uint32_t* __restrict__ n_occ)
{
    using CT = typename Stage<PREC>::T;
    using Real = typename std::conditional<PREC == 0, double, float>::type;
    constexpr int CAP = Stage<PREC>::CAP;
    __shared__ CT s_stage[FL_WAVES][CAP];
    __shared__ uint8_t s_type[FL_WAVES][MULTI ? CAP : 1];
    __shared__ uint16_t s_list[FL_WAVES][FL_LIST][WAVE];

    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    CT* stage = s_stage[w];
    const uint32_t M = *n_occ;
    uint32_t inter = 0, cand = 0;

    // wave q of the (XCD-renumbered) grid takes occupied voxels q, q + W, q + 2W, ...
    const uint32_t nwaves = gridDim.x * FL_WAVES;
    const uint32_t q0 = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * FL_WAVES + w);
    for (uint32_t o = q0; o < M; o += nwaves) {
        const uint32_t vox = __builtin_amdgcn_readfirstlane(occ[o]);
        const int kx = (int)(vox % (uint32_t)P.nx);
        const int ky = (int)((vox / (uint32_t)P.nx) % (uint32_t)P.ny);
        const int kz = (int)(vox / ((uint32_t)P.nx * (uint32_t)P.ny));
        const int x0 = kx > 0 ? kx - 1 : 0;
        const int x1 = kx < P.nx - 1 ? kx + 1 : P.nx - 1;
        // the 9 rows in (dz, dy) order; rows outside the grid are empty
        uint32_t rb[9], pre[10];
        pre[0] = 0;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int y = ky + (q % 3) - 1, z = kz + (q / 3) - 1;
            uint32_t b = 0, e = 0;
            if (y >= 0 && y < P.ny && z >= 0 && z < P.nz) {
                const uint32_t row = (uint32_t)P.nx * ((uint32_t)y + (uint32_t)P.ny * (uint32_t)z);
                b = a.voxel_start[row + x0];
                e = a.voxel_start[row + x1 + 1];
            }
            rb[q] = b;
            pre[q + 1] = pre[q] + (e - b);
        }
        const uint32_t C = pre[9];
        const uint32_t vb = a.voxel_start[vox], k = a.voxel_start[vox + 1] - vb;

        for (uint32_t t0 = 0; t0 < k; t0 += WAVE) {
            const uint32_t r = min((uint32_t)WAVE, k - t0);
            const uint32_t t = (uint32_t)lane % r, s = (uint32_t)lane / r;
            const uint32_t St = (uint32_t)WAVE / r + (t < (uint32_t)WAVE % r ? 1u : 0u);
            const uint32_t i = vb + t0 + t;
            CT me;
            if constexpr (PREC == 0) {
                me = make_double4(a.XS[0][i], a.XS[1][i], a.XS[2][i], a.R[i]);
            } else {
                me = a.SH[i];
            }
            const int ti = MULTI ? a.T[i] : 0;
            Real acc[3] = {0, 0, 0}, cmp[3] = {0, 0, 0};
            uint32_t cnt = 0;

            // evaluate this lane's listed candidates in order, then empty the list
            auto flush = [&]() {
                for (uint32_t q = 0; q < (uint32_t)FL_LIST; ++q) {
                    if (!__any(q < cnt)) break;
                    if (q < cnt) {
                        const uint32_t m = s_list[w][q][lane];
                        const CT c = stage[m];
                        if constexpr (PREC == 0) {
                            const double cadh = MULTI ? a.cadh[ti * P.n_types + s_type[w][m]] : P.c_adh0;
                            pair64(me.x, me.y, me.z, me.w, c.x, c.y, c.z, c.w, P.alpha, P.c_rep, cadh,
                                   acc[0], acc[1], acc[2]);
                        } else {
                            const float cadh = MULTI ? a.cadh_f[ti * P.n_types + s_type[w][m]] : P.c_adh0_f;
                            pair32<PREC == 2>(me.x, me.y, me.z, me.w, c, P.alpha_f, P.c_rep_f, cadh, acc, cmp);
                        }
                    }
                }
                cnt = 0;
            };

            for (uint32_t cb = 0; cb < C; cb += CAP) {
                const uint32_t len = min((uint32_t)CAP, C - cb);
                wave_sync();
                for (uint32_t f = lane; f < len; f += WAVE) {
                    const uint32_t ff = cb + f;
                    uint32_t g = ff + rb[0];
#pragma unroll
                    for (int q = 1; q < 9; ++q)
                        if (ff >= pre[q]) g = ff - pre[q] + rb[q];
                    if constexpr (PREC == 0) {
                        stage[f] = make_double4(a.XS[0][g], a.XS[1][g], a.XS[2][g], a.R[g]);
                    } else {
                        stage[f] = a.SH[g];
                    }
                    if (MULTI) s_type[w][f] = (uint8_t)a.T[g];
                }
                wave_sync();
                for (uint32_t m = s; m < len; m += St) {
                    bool in;
                    if constexpr (PREC == 0)
                        in = in_range64(me, stage[m], P.alpha);
                    else
                        in = in_range32(me, stage[m], P.alpha_f);
                    if (in) {
                        s_list[w][cnt][lane] = (uint16_t)m;
                        ++cnt;
                    }
                    if (__any(cnt == (uint32_t)FL_LIST)) {
                        inter += cnt;
                        flush();
                    }
                }
                inter += cnt;
                flush();
            }
            // combine the slices of each target in slice order
            wave_sync();
            Real* part = reinterpret_cast<Real*>(stage);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                part[lane * 6 + c] = acc[c];
                part[lane * 6 + 3 + c] = cmp[c];
            }
            wave_sync();
            if (s == 0) {
                Real tot[3] = {0, 0, 0}, tc[3] = {0, 0, 0};
                for (uint32_t q = 0; q < St; ++q) {
                    const uint32_t l = t + q * r;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const Real term = part[l * 6 + c] - part[l * 6 + 3 + c];
                        if (PREC == 2) {
                            const Real y = term - tc[c];
                            const Real tt = tot[c] + y;
                            tc[c] = (tt - tot[c]) - y;
                            tot[c] = tt;
                        } else {
                            tot[c] += term;
                        }
                    }
                }
                cand += C - 1;
                const double xs[3] = {a.XS[0][i], a.XS[1][i], a.XS[2][i]};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double v = (double)tot[c];
                    const double vp = a.euler ? v : (double)a.VP[c][i];
                    const double xn = xs[c] + P.dt * (1.5 * v - 0.5 * vp);
                    a.X[c][i] = reflect(xn, (&P.lo[0])[c], (&P.hi[0])[c]);
                    a.VP[c][i] = (VPT)v;
                }
            }
            wave_sync();
        }
    }
    add_stats(a.stats, inter, cand);
}

// read_state: voxel order -> id order, interleaved xyz.
template <typename VPT>
__global__ __launch_bounds__(BLOCK) void k_unpermute(uint32_t n, const uint32_t* __restrict__ id,
                                                     const double* __restrict__ x0,
                                                     const double* __restrict__ x1,
                                                     const double* __restrict__ x2,
                                                     const VPT* __restrict__ v0,
                                                     const VPT* __restrict__ v1,
                                                     const VPT* __restrict__ v2,
                                                     double* __restrict__ pos,
                                                     double* __restrict__ vel)
{
    uint32_t s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= n) return;
    uint32_t k = id[s];
    pos[3 * k + 0] = x0[s];
    pos[3 * k + 1] = x1[s];
    pos[3 * k + 2] = x2[s];
    vel[3 * k + 0] = (double)v0[s];
    vel[3 * k + 1] = (double)v1[s];
    vel[3 * k + 2] = (double)v2[s];
}

// ------------------------------------------------------------------------ host side

inline uint32_t blocks_for(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

struct Layout {
    size_t X[3], XS[3], R[2], T[2], ID[2], VP[2][3], SH, vid_cur, off, tmp_key, tmp_src,
        vid_sorted, count, start, occ, n_occ, tsum, stats, cadh, cadh_f, stage;
    size_t total;
};

bool is_fp32(const MechParams& p) { return p.precision != MECH_FP64; }

Layout make_layout(const MechParams& p, int64_t n, uint64_t V)
{
    Layout L{};
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        size_t o = cur;
        cur += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    const size_t vpb = is_fp32(p) ? sizeof(float) : sizeof(double);
    for (int c = 0; c < 3; ++c) L.X[c] = take(nn * 8);
    for (int c = 0; c < 3; ++c) L.XS[c] = take(nn * 8);
    for (int k = 0; k < 2; ++k) {
        L.R[k] = take(nn * 8);
        L.T[k] = take(nn * 4);
        L.ID[k] = take(nn * 4);
        for (int c = 0; c < 3; ++c) L.VP[k][c] = take(nn * vpb);
    }
    L.SH = is_fp32(p) ? take(nn * 16) : 0;
    L.vid_cur = take(nn * 4);
    L.off = take(nn * 4);
    L.tmp_key = take(nn * 4);
    L.tmp_src = take(nn * 4);
    L.vid_sorted = take(nn * 4);
    L.count = take(V * 4);
    L.start = take((V + 1) * 4);
    L.occ = take(V * 4);
    L.n_occ = take(16);
    L.tsum = take((size_t)blocks_for(V, SCAN_TILE) * 8);
    L.stats = take(STAT_SLOTS * 16);
    L.cadh = take(64 * 8);
    L.cadh_f = take(64 * 4);
    L.stage = take(nn * 48);
    L.total = cur;
    return L;
}

int validate(const MechParams* p, int64_t n, int32_t dims[3])
{
    if (!p) return fail(MECH_E_INVALID, "params is NULL");
    if (p->abi_version != MECH_ABI_VERSION)
        return fail(MECH_E_INVALID, "abi_version %d, library is %d", p->abi_version, MECH_ABI_VERSION);
    if (p->precision < MECH_FP64 || p->precision > MECH_FP32_KAHAN)
        return fail(MECH_E_INVALID, "precision %d unknown", p->precision);
    if (p->ab2_start != MECH_AB2_ZERO_HISTORY && p->ab2_start != MECH_AB2_EULER_START)
        return fail(MECH_E_INVALID, "ab2_start %d unknown", p->ab2_start);
    if (p->flags & ~(MECH_FLAG_NO_GRAPH | MECH_FORCE_KERNEL_MASK))
        return fail(MECH_E_INVALID, "unknown flags 0x%x", p->flags);
    {
        const int k = p->flags & MECH_FORCE_KERNEL_MASK;
        if (k & (k - 1)) return fail(MECH_E_INVALID, "at most one force-kernel flag may be set");
    }
    if (p->reserved != 0) return fail(MECH_E_INVALID, "reserved field must be 0");
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(MECH_E_INVALID, "n_cells %lld out of range", (long long)n);
    if (!(std::isfinite(p->voxel_size) && p->voxel_size > 0))
        return fail(MECH_E_INVALID, "voxel_size must be finite and > 0");
    if (!(std::isfinite(p->dt) && p->dt > 0)) return fail(MECH_E_INVALID, "dt must be finite and > 0");
    if (!(std::isfinite(p->c_rep) && p->c_rep >= 0)) return fail(MECH_E_INVALID, "c_rep must be finite and >= 0");
    if (!(std::isfinite(p->rel_adh_distance) && p->rel_adh_distance >= 1.0))
        return fail(MECH_E_INVALID, "rel_adh_distance must be finite and >= 1");
    if (p->n_types < 1 || p->n_types > 8) return fail(MECH_E_INVALID, "n_types %d not in 1..8", p->n_types);
    for (int i = 0; i < p->n_types; ++i)
        for (int j = 0; j < p->n_types; ++j) {
            double a = p->c_adh[i * p->n_types + j], b = p->c_adh[j * p->n_types + i];
            if (!std::isfinite(a) || a < 0) return fail(MECH_E_INVALID, "c_adh[%d][%d] must be finite and >= 0", i, j);
            if (a != b) return fail(MECH_E_INVALID, "c_adh is not symmetric at [%d][%d]", i, j);
        }
    uint64_t V = 1;
    for (int a = 0; a < 3; ++a) {
        double lo = p->domain_lo[a], hi = p->domain_hi[a];
        if (!(std::isfinite(lo) && std::isfinite(hi) && hi >= lo))
            return fail(MECH_E_INVALID, "domain axis %d: need finite lo <= hi", a);
        double cells = std::ceil((hi - lo) / p->voxel_size);
        if (cells > 2147483647.0) return fail(MECH_E_INVALID, "too many voxels on axis %d", a);
        dims[a] = std::max(1, (int)cells);
        V *= (uint64_t)dims[a];
    }
    if (V >= (uint64_t(1) << 31)) return fail(MECH_E_INVALID, "grid of %llu voxels is too large", (unsigned long long)V);
    return MECH_OK;
}

int validate_cells(const MechParams* p, int64_t n, const double* pos, const double* radius,
                   const int32_t* type, const double* vprev)
{
    if (n > 0 && (!pos || !radius)) return fail(MECH_E_INVALID, "pos and radius are required");
    double rmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double r = radius[i];
        if (!(std::isfinite(r) && r > 0)) return fail(MECH_E_INVALID, "radius[%lld] must be finite and > 0", (long long)i);
        rmax = std::max(rmax, r);
        for (int a = 0; a < 3; ++a) {
            double x = pos[3 * i + a];
            if (!std::isfinite(x)) return fail(MECH_E_INVALID, "pos[%lld] is not finite", (long long)i);
            if (x < p->domain_lo[a] || x > p->domain_hi[a])
                return fail(MECH_E_OUT_OF_DOMAIN, "cell %lld lies outside the domain on axis %d", (long long)i, a);
            if (vprev && !std::isfinite(vprev[3 * i + a]))
                return fail(MECH_E_INVALID, "prev_velocity[%lld] is not finite", (long long)i);
        }
        if (type && (type[i] < 0 || type[i] >= p->n_types))
            return fail(MECH_E_INVALID, "type[%lld] = %d not in [0, %d)", (long long)i, type[i], p->n_types);
    }
    // every interacting pair must lie in the 27 voxels around a cell
    if (p->voxel_size < p->rel_adh_distance * 2.0 * rmax)
        return fail(MECH_E_VOXEL_TOO_SMALL, "voxel_size %.17g < %.17g (rel_adh_distance * 2 * max radius)",
                    p->voxel_size, p->rel_adh_distance * 2.0 * rmax);
    return MECH_OK;
}

}  // namespace

struct MechPopulation {
    MechParams prm;
    int device = 0;
    int64_t n = 0;
    int32_t dims[3] = {1, 1, 1};
    uint32_t V = 1, n_tiles = 1;
    uint32_t force_grid = 1024;  // workgroups of the persistent force kernel
    GridArgs grid{};
    PhysArgs phys{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* arena = nullptr;
    bool own_arena = false;
    Layout L{};
    int parity = 0;
    int64_t steps = 0;
    bool euler_pending = false;
    bool graphs_ready = false;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};

    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(arena + off); }
};

namespace {

template <typename VPT>
void enqueue_binning(MechPopulation* P)
{
    const uint32_t n = (uint32_t)P->n;
    const Layout& L = P->L;
    const int cur = P->parity, nxt = cur ^ 1;
    const uint32_t nb = blocks_for(n, BLOCK);
    hipLaunchKernelGGL(k_bin, dim3(nb), dim3(BLOCK), 0, P->stream, P->at<double>(L.X[0]),
                       P->at<double>(L.X[1]), P->at<double>(L.X[2]), n, P->grid,
                       P->at<uint32_t>(L.count), P->at<uint32_t>(L.vid_cur), P->at<uint32_t>(L.off));
    hipLaunchKernelGGL(k_scan_reduce, dim3(P->n_tiles), dim3(BLOCK), 0, P->stream,
                       P->at<uint32_t>(L.count), P->V, P->at<uint64_t>(L.tsum));
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(BLOCK), 0, P->stream, P->at<uint64_t>(L.tsum),
                       P->n_tiles, P->at<uint32_t>(L.start), P->V, P->at<uint32_t>(L.n_occ));
    hipLaunchKernelGGL(k_scan_down, dim3(P->n_tiles), dim3(BLOCK), 0, P->stream,
                       P->at<uint32_t>(L.count), P->V, P->at<uint64_t>(L.tsum),
                       P->at<uint32_t>(L.start), P->at<uint32_t>(L.occ));
    hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(BLOCK), 0, P->stream, n, P->at<uint32_t>(L.vid_cur),
                       P->at<uint32_t>(L.off), P->at<uint32_t>(L.start), P->at<uint32_t>(L.ID[cur]),
                       P->at<uint32_t>(L.tmp_key), P->at<uint32_t>(L.tmp_src));
    GatherArgs<VPT> g{};
    for (int c = 0; c < 3; ++c) {
        g.X[c] = P->at<double>(L.X[c]);
        g.XS[c] = P->at<double>(L.XS[c]);
        g.VP_cur[c] = P->at<VPT>(L.VP[cur][c]);
        g.VP_new[c] = P->at<VPT>(L.VP[nxt][c]);
    }
    g.R_cur = P->at<double>(L.R[cur]);
    g.R_new = P->at<double>(L.R[nxt]);
    g.T_cur = P->at<int32_t>(L.T[cur]);
    g.T_new = P->at<int32_t>(L.T[nxt]);
    g.ID_new = P->at<uint32_t>(L.ID[nxt]);
    g.SH = is_fp32(P->prm) ? P->at<float4>(L.SH) : nullptr;
    g.vid_cur = P->at<uint32_t>(L.vid_cur);
    g.tmp_key = P->at<uint32_t>(L.tmp_key);
    g.tmp_src = P->at<uint32_t>(L.tmp_src);
    g.voxel_start = P->at<uint32_t>(L.start);
    g.vid_sorted = P->at<uint32_t>(L.vid_sorted);
    hipLaunchKernelGGL(k_rank_gather<VPT>, dim3(nb), dim3(BLOCK), 0, P->stream, n, g);
}

template <int PREC, typename VPT>
void enqueue_force(MechPopulation* P, int parity_after_sort, int euler)
{
    const uint32_t n = (uint32_t)P->n;
    const Layout& L = P->L;
    const int p = parity_after_sort;
    ForceArgs<VPT> a{};
    for (int c = 0; c < 3; ++c) {
        a.XS[c] = P->at<double>(L.XS[c]);
        a.X[c] = P->at<double>(L.X[c]);
        a.VP[c] = P->at<VPT>(L.VP[p][c]);
    }
    a.R = P->at<double>(L.R[p]);
    a.T = P->at<int32_t>(L.T[p]);
    a.SH = is_fp32(P->prm) ? P->at<float4>(L.SH) : nullptr;
    a.vid_sorted = P->at<uint32_t>(L.vid_sorted);
    a.voxel_start = P->at<uint32_t>(L.start);
    a.cadh = P->at<double>(L.cadh);
    a.cadh_f = P->at<float>(L.cadh_f);
    a.stats = P->at<unsigned long long>(L.stats);
    a.euler = euler;
    if (P->prm.flags & MECH_FLAG_SIMPLE_FORCE) {
        const uint32_t nb = blocks_for(n, BLOCK);
        if (P->prm.n_types > 1)
            hipLaunchKernelGGL((k_force_rows<PREC, true, VPT>), dim3(nb), dim3(BLOCK), 0, P->stream, n, P->phys, a);
        else
            hipLaunchKernelGGL((k_force_rows<PREC, false, VPT>), dim3(nb), dim3(BLOCK), 0, P->stream, n, P->phys, a);
        return;
    }
    if (!(P->prm.flags & MECH_FLAG_VOXEL_FORCE)) {
        const uint32_t nb = blocks_for(n, BLOCK);
        if (P->prm.n_types > 1)
            hipLaunchKernelGGL((k_force_cells<PREC, true, VPT>), dim3(nb), dim3(BLOCK), 0, P->stream, n, P->phys, a);
        else
            hipLaunchKernelGGL((k_force_cells<PREC, false, VPT>), dim3(nb), dim3(BLOCK), 0, P->stream, n, P->phys, a);
        return;
    }
    // persistent grid of fixed size (graph-safe); waves walk the occupied-voxel list
    const uint32_t* occ = P->at<uint32_t>(L.occ);
    const uint32_t* m = P->at<uint32_t>(L.n_occ);
    if (P->prm.n_types > 1)
        hipLaunchKernelGGL((k_force_lds<PREC, true, VPT>), dim3(P->force_grid), dim3(FL_WAVES * WAVE), 0,
                           P->stream, P->phys, a, occ, m);
    else
        hipLaunchKernelGGL((k_force_lds<PREC, false, VPT>), dim3(P->force_grid), dim3(FL_WAVES * WAVE), 0,
                           P->stream, P->phys, a, occ, m);
}

// One full step a1..a7 from the current parity; flips nothing on the host.
void enqueue_step(MechPopulation* P, int parity, int euler)
{
    const int saved = P->parity;
    P->parity = parity;
    switch (P->prm.precision) {
    case MECH_FP64:
        enqueue_binning<double>(P);
        enqueue_force<0, double>(P, parity ^ 1, euler);
        break;
    case MECH_FP32:
        enqueue_binning<float>(P);
        enqueue_force<1, float>(P, parity ^ 1, euler);
        break;
    default:
        enqueue_binning<float>(P);
        enqueue_force<2, float>(P, parity ^ 1, euler);
        break;
    }
    P->parity = saved;
}

int sync_check(MechPopulation* P)
{
    HIP_TRY(hipStreamSynchronize(P->stream));
    HIP_TRY(hipGetLastError());
    return MECH_OK;
}

int build_graphs(MechPopulation* P)
{
    for (int p = 0; p < 2; ++p) {
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal));
        enqueue_step(P, p, 0);
        hipError_t e = hipStreamEndCapture(P->stream, &g);
        if (e != hipSuccess) return fail(MECH_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&P->gexec[p], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(MECH_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    P->graphs_ready = true;
    return MECH_OK;
}

void release(MechPopulation* P)
{
    if (!P) return;
    (void)hipSetDevice(P->device);
    if (P->stream) (void)hipStreamSynchronize(P->stream);
    for (int p = 0; p < 2; ++p)
        if (P->gexec[p]) (void)hipGraphExecDestroy(P->gexec[p]);
    if (P->own_arena && P->arena) (void)hipFree(P->arena);
    if (P->own_stream && P->stream) (void)hipStreamDestroy(P->stream);
    delete P;
}

int create_impl(const MechParams* params, int64_t n, const double* pos, const double* radius,
                const int32_t* type, const double* vprev, void* stream, void* workspace,
                int64_t ws_bytes, MechPopulation** out)
{
    if (!out) return fail(MECH_E_INVALID, "out is NULL");
    *out = nullptr;
    int32_t dims[3];
    int rc = validate(params, n, dims);
    if (rc) return rc;
    rc = validate_cells(params, n, pos, radius, type, vprev);
    if (rc) return rc;

    MechPopulation* P = new MechPopulation();
    P->prm = *params;
    P->n = n;
    HIP_TRY(hipGetDevice(&P->device));
    for (int a = 0; a < 3; ++a) P->dims[a] = dims[a];
    P->V = (uint32_t)((uint64_t)dims[0] * dims[1] * dims[2]);
    P->n_tiles = blocks_for(P->V, SCAN_TILE);
    for (int a = 0; a < 3; ++a) {
        P->grid.lo[a] = params->domain_lo[a];
        P->grid.n[a] = dims[a];
        P->phys.lo[a] = params->domain_lo[a];
        P->phys.hi[a] = params->domain_hi[a];
    }
    P->grid.inv_h = 1.0 / params->voxel_size;
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device) != hipSuccess || cus < 1)
            cus = 256;
        P->force_grid = (uint32_t)cus * 4u;  // a few resident workgroups per CU
    }
    P->grid.V = P->V;
    P->phys.dt = params->dt;
    P->phys.c_rep = params->c_rep;
    P->phys.alpha = params->rel_adh_distance;
    P->phys.c_adh0 = params->c_adh[0];
    P->phys.c_rep_f = (float)params->c_rep;
    P->phys.alpha_f = (float)params->rel_adh_distance;
    P->phys.c_adh0_f = (float)params->c_adh[0];
    {
        double rmax = 0.0;
        for (int64_t k = 0; k < n; ++k) rmax = std::max(rmax, radius[k]);
        P->phys.r_max = rmax;
        P->phys.r_max_f = (float)rmax;
    }
    P->phys.n_types = params->n_types;
    P->phys.nx = dims[0];
    P->phys.ny = dims[1];
    P->phys.nz = dims[2];
    P->L = make_layout(*params, n, P->V);
    P->euler_pending = (params->ab2_start == MECH_AB2_EULER_START) && vprev == nullptr;

    auto bail = [&](int code) {
        release(P);
        return code;
    };
    if (stream) {
        P->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(MECH_E_DEVICE, "hipStreamCreate failed"));
        P->own_stream = true;
    }
    if (workspace) {
        if (ws_bytes < (int64_t)P->L.total)
            return bail(fail(MECH_E_NOMEM, "workspace of %lld bytes < %zu needed", (long long)ws_bytes, P->L.total));
        if (((uintptr_t)workspace & 255u) != 0)
            return bail(fail(MECH_E_INVALID, "workspace must be 256-byte aligned"));
        P->arena = (char*)workspace;
    } else {
        if (hipMalloc(&P->arena, P->L.total) != hipSuccess) {
            P->arena = nullptr;
            (void)hipGetLastError();
            return bail(fail(MECH_E_NOMEM, "hipMalloc of %zu bytes failed", P->L.total));
        }
        P->own_arena = true;
    }

    // host-side staging: structure of arrays, v_prev in the variant's precision
    const size_t nn = (size_t)n;
    std::vector<double> soa(3 * nn);
    std::vector<uint32_t> ids(nn);
    std::vector<int32_t> tz;
    for (size_t i = 0; i < nn; ++i) {
        for (int c = 0; c < 3; ++c) soa[c * nn + i] = pos[3 * i + c];
        ids[i] = (uint32_t)i;
    }
    const Layout& L = P->L;
    hipStream_t s = P->stream;
    int e = 0;
    auto H2D = [&](size_t off, const void* src, size_t bytes) {
        if (bytes && hipMemcpyAsync(P->arena + off, src, bytes, hipMemcpyHostToDevice, s) != hipSuccess) e = 1;
    };
    for (int c = 0; c < 3; ++c) H2D(L.X[c], soa.data() + c * nn, nn * 8);
    H2D(L.R[0], radius, nn * 8);
    if (type) {
        H2D(L.T[0], type, nn * 4);
    } else {
        tz.assign(nn, 0);
        H2D(L.T[0], tz.data(), nn * 4);
    }
    H2D(L.ID[0], ids.data(), nn * 4);
    std::vector<double> vp64;
    std::vector<float> vp32;
    if (is_fp32(*params)) {
        vp32.assign(3 * nn, 0.f);
        if (vprev)
            for (size_t i = 0; i < nn; ++i)
                for (int c = 0; c < 3; ++c) vp32[c * nn + i] = (float)vprev[3 * i + c];
        for (int c = 0; c < 3; ++c) H2D(L.VP[0][c], vp32.data() + c * nn, nn * 4);
    } else {
        vp64.assign(3 * nn, 0.0);
        if (vprev)
            for (size_t i = 0; i < nn; ++i)
                for (int c = 0; c < 3; ++c) vp64[c * nn + i] = vprev[3 * i + c];
        for (int c = 0; c < 3; ++c) H2D(L.VP[0][c], vp64.data() + c * nn, nn * 8);
    }
    double cd[64];
    float cf[64];
    for (int k = 0; k < 64; ++k) {
        cd[k] = params->c_adh[k];
        cf[k] = (float)params->c_adh[k];
    }
    H2D(L.cadh, cd, sizeof cd);
    H2D(L.cadh_f, cf, sizeof cf);
    if (e) return bail(fail(MECH_E_DEVICE, "host to device copy failed"));
    if (hipMemsetAsync(P->arena + L.count, 0, (size_t)P->V * 4, s) != hipSuccess ||
        hipMemsetAsync(P->arena + L.stats, 0, STAT_SLOTS * 16, s) != hipSuccess ||
        hipMemsetAsync(P->arena + L.start, 0, ((size_t)P->V + 1) * 4, s) != hipSuccess ||
        hipMemsetAsync(P->arena + L.n_occ, 0, 16, s) != hipSuccess)
        return bail(fail(MECH_E_DEVICE, "hipMemsetAsync failed"));

    // initial binning (parity 0 -> 1); positions in voxel order become the state
    if (n > 0) {
        P->parity = 0;
        if (is_fp32(*params))
            enqueue_binning<float>(P);
        else
            enqueue_binning<double>(P);
        hipLaunchKernelGGL(k_copy_positions, dim3(blocks_for(n, BLOCK)), dim3(BLOCK), 0, s, (uint32_t)n,
                           P->at<double>(L.XS[0]), P->at<double>(L.XS[1]), P->at<double>(L.XS[2]),
                           P->at<double>(L.X[0]), P->at<double>(L.X[1]), P->at<double>(L.X[2]));
        P->parity = 1;
    }
    rc = sync_check(P);
    if (rc) return bail(rc);
    *out = P;
    return MECH_OK;
}

}  // namespace

// ------------------------------------------------------------------------ C ABI

extern "C" {

const char* mech_last_error(void) { return g_err.c_str(); }

int32_t mech_abi_version(void) { return MECH_ABI_VERSION; }

int32_t mech_device_count(void)
{
    int c = 0;
    if (hipGetDeviceCount(&c) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return c;
}

int64_t population_workspace_bytes(const MechParams* params, int64_t n_cells)
{
    int32_t dims[3];
    int rc = validate(params, n_cells, dims);
    if (rc) return rc;
    uint64_t V = (uint64_t)dims[0] * dims[1] * dims[2];
    return (int64_t)make_layout(*params, n_cells, V).total;
}

int create_population(const MechParams* params, int64_t n_cells, const double* pos,
                      const double* radius, const int32_t* type, const double* prev_velocity,
                      void* hip_stream, MechPopulation** out)
{
    return create_impl(params, n_cells, pos, radius, type, prev_velocity, hip_stream, nullptr, 0, out);
}

int create_population_in(const MechParams* params, int64_t n_cells, const double* pos,
                         const double* radius, const int32_t* type, const double* prev_velocity,
                         void* hip_stream, void* workspace, int64_t workspace_bytes,
                         MechPopulation** out)
{
    if (!workspace) {
        if (out) *out = nullptr;
        return fail(MECH_E_INVALID, "workspace is NULL");
    }
    return create_impl(params, n_cells, pos, radius, type, prev_velocity, hip_stream, workspace,
                       workspace_bytes, out);
}

int step_mechanics(MechPopulation* P, int64_t n_steps)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    if (n_steps < 0) return fail(MECH_E_INVALID, "n_steps must be >= 0");
    HIP_TRY(hipSetDevice(P->device));
    const bool eager = (P->prm.flags & MECH_FLAG_NO_GRAPH) != 0;
    for (int64_t k = 0; k < n_steps; ++k) {
        if (P->n > 0) {
            if (P->euler_pending || eager) {
                enqueue_step(P, P->parity, P->euler_pending ? 1 : 0);
            } else {
                if (!P->graphs_ready) {
                    int rc = build_graphs(P);
                    if (rc) return rc;
                }
                HIP_TRY(hipGraphLaunch(P->gexec[P->parity], P->stream));
            }
            HIP_TRY(hipGetLastError());
            P->parity ^= 1;
        }
        P->euler_pending = false;
        ++P->steps;
    }
    return MECH_OK;
}

int profile_step(MechPopulation* P, int64_t n_steps, double* phase_ms)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    if (!phase_ms || n_steps < 1) return fail(MECH_E_INVALID, "need phase_ms and n_steps >= 1");
    HIP_TRY(hipSetDevice(P->device));
    phase_ms[0] = phase_ms[1] = 0.0;
    if (P->n == 0) {
        P->steps += n_steps;
        return MECH_OK;
    }
    hipEvent_t ev[3];
    for (int k = 0; k < 3; ++k) HIP_TRY(hipEventCreate(&ev[k]));
    double acc[2] = {0.0, 0.0};
    int rc = MECH_OK;
    for (int64_t s = 0; s < n_steps && rc == MECH_OK; ++s) {
        const int euler = P->euler_pending ? 1 : 0;
        const int p = P->parity;
        (void)hipEventRecord(ev[0], P->stream);
        switch (P->prm.precision) {
        case MECH_FP64:
            enqueue_binning<double>(P);
            (void)hipEventRecord(ev[1], P->stream);
            enqueue_force<0, double>(P, p ^ 1, euler);
            break;
        case MECH_FP32:
            enqueue_binning<float>(P);
            (void)hipEventRecord(ev[1], P->stream);
            enqueue_force<1, float>(P, p ^ 1, euler);
            break;
        default:
            enqueue_binning<float>(P);
            (void)hipEventRecord(ev[1], P->stream);
            enqueue_force<2, float>(P, p ^ 1, euler);
            break;
        }
        (void)hipEventRecord(ev[2], P->stream);
        P->parity ^= 1;
        P->euler_pending = false;
        ++P->steps;
        rc = sync_check(P);
        float t0 = 0.f, t1 = 0.f;
        if (rc == MECH_OK && (hipEventElapsedTime(&t0, ev[0], ev[1]) != hipSuccess ||
                              hipEventElapsedTime(&t1, ev[1], ev[2]) != hipSuccess))
            rc = fail(MECH_E_DEVICE, "hipEventElapsedTime failed");
        acc[0] += t0;
        acc[1] += t1;
    }
    for (int k = 0; k < 3; ++k) (void)hipEventDestroy(ev[k]);
    if (rc) return rc;
    phase_ms[0] = acc[0] / (double)n_steps;
    phase_ms[1] = acc[1] / (double)n_steps;
    return MECH_OK;
}

int read_state(MechPopulation* P, double* pos, double* vel, int64_t n_cells)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    if (!pos) return fail(MECH_E_INVALID, "pos is NULL");
    if (n_cells != P->n) return fail(MECH_E_INVALID, "n_cells %lld != population size %lld", (long long)n_cells, (long long)P->n);
    HIP_TRY(hipSetDevice(P->device));
    if (P->n == 0) return MECH_OK;
    const Layout& L = P->L;
    const int p = P->parity;
    const uint32_t n = (uint32_t)P->n;
    double* st = P->at<double>(L.stage);
    if (is_fp32(P->prm))
        hipLaunchKernelGGL(k_unpermute<float>, dim3(blocks_for(n, BLOCK)), dim3(BLOCK), 0, P->stream, n,
                           P->at<uint32_t>(L.ID[p]), P->at<double>(L.X[0]), P->at<double>(L.X[1]),
                           P->at<double>(L.X[2]), P->at<float>(L.VP[p][0]), P->at<float>(L.VP[p][1]),
                           P->at<float>(L.VP[p][2]), st, st + 3 * (size_t)n);
    else
        hipLaunchKernelGGL(k_unpermute<double>, dim3(blocks_for(n, BLOCK)), dim3(BLOCK), 0, P->stream, n,
                           P->at<uint32_t>(L.ID[p]), P->at<double>(L.X[0]), P->at<double>(L.X[1]),
                           P->at<double>(L.X[2]), P->at<double>(L.VP[p][0]), P->at<double>(L.VP[p][1]),
                           P->at<double>(L.VP[p][2]), st, st + 3 * (size_t)n);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(pos, st, 24 * (size_t)n, hipMemcpyDeviceToHost, P->stream));
    if (vel) HIP_TRY(hipMemcpyAsync(vel, st + 3 * (size_t)n, 24 * (size_t)n, hipMemcpyDeviceToHost, P->stream));
    int rc = sync_check(P);
    if (rc) return rc;
    for (size_t i = 0; i < 3 * (size_t)n; ++i)
        if (!std::isfinite(pos[i]) || (vel && !std::isfinite(vel[i])))
            return fail(MECH_E_NONFINITE, "state holds a non-finite value at cell %zu", i / 3);
    return MECH_OK;
}

int read_binning(MechPopulation* P, uint32_t* voxel_of_cell, uint32_t* voxel_start,
                 uint32_t* sorted_ids, uint32_t* occ, int64_t* n_occ, int64_t* n_voxels)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    HIP_TRY(hipSetDevice(P->device));
    int rc = sync_check(P);
    if (rc) return rc;
    const Layout& L = P->L;
    const size_t n = (size_t)P->n;
    if (n_voxels) *n_voxels = P->V;
    uint32_t m = 0;
    if (n > 0) HIP_TRY(hipMemcpy(&m, P->arena + L.n_occ, 4, hipMemcpyDeviceToHost));
    if (n_occ) *n_occ = m;
    if (voxel_start) {
        if (n > 0)
            HIP_TRY(hipMemcpy(voxel_start, P->arena + L.start, ((size_t)P->V + 1) * 4, hipMemcpyDeviceToHost));
        else
            std::memset(voxel_start, 0, ((size_t)P->V + 1) * 4);
    }
    if (occ && m) HIP_TRY(hipMemcpy(occ, P->arena + L.occ, (size_t)m * 4, hipMemcpyDeviceToHost));
    if (n == 0) return MECH_OK;
    std::vector<uint32_t> ids(n), vs(n);
    HIP_TRY(hipMemcpy(ids.data(), P->arena + L.ID[P->parity], n * 4, hipMemcpyDeviceToHost));
    if (sorted_ids) std::memcpy(sorted_ids, ids.data(), n * 4);
    if (voxel_of_cell) {
        HIP_TRY(hipMemcpy(vs.data(), P->arena + L.vid_sorted, n * 4, hipMemcpyDeviceToHost));
        for (size_t s = 0; s < n; ++s) voxel_of_cell[ids[s]] = vs[s];
    }
    return MECH_OK;
}

int read_stats(MechPopulation* P, int64_t* steps, int64_t* interactions, int64_t* candidates)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    HIP_TRY(hipSetDevice(P->device));
    int rc = sync_check(P);
    if (rc) return rc;
    std::vector<unsigned long long> slots(2 * STAT_SLOTS);
    HIP_TRY(hipMemcpy(slots.data(), P->arena + P->L.stats, slots.size() * 8, hipMemcpyDeviceToHost));
    unsigned long long st[2] = {0, 0};
    for (uint32_t k = 0; k < STAT_SLOTS; ++k) {
        st[0] += slots[2 * k];
        st[1] += slots[2 * k + 1];
    }
    if (steps) *steps = P->steps;
    if (interactions) *interactions = (int64_t)st[0];
    if (candidates) *candidates = (int64_t)st[1];
    return MECH_OK;
}

int population_info(MechPopulation* P, int64_t* n_cells, int32_t dims[3])
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    if (n_cells) *n_cells = P->n;
    if (dims)
        for (int a = 0; a < 3; ++a) dims[a] = P->dims[a];
    return MECH_OK;
}

void* population_stream(MechPopulation* P) { return P ? (void*)P->stream : nullptr; }

int destroy_population(MechPopulation* P)
{
    if (!P) return MECH_OK;
    (void)hipSetDevice(P->device);
    hipError_t e = P->stream ? hipStreamSynchronize(P->stream) : hipSuccess;
    release(P);
    if (e != hipSuccess) return fail(MECH_E_DEVICE, "stream error at destroy: %s", hipGetErrorString(e));
    return MECH_OK;
}

}  // extern "C"
