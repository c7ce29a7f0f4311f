// mech.hip -- gfx950 kernels and C-ABI runtime of the agent-mechanics step (libmech.so).
//
// One step, all on the device, on the batch's stream:
//   k_bin          a1+a2  storage bin of every cell (its voxel, cut into XSUB slabs along x;
//                         FP64 key) and an integer-atomic histogram, one atomic per run of
//                         equal bins in a wave; a workgroup also does the step's
//                         per-simulation bookkeeping (step counters, Euler start), and on
//                         large grids an extra first one cuts the force kernel's XCD runs
//                         from the last launch's measured work
//   k_scan_reduce  a3     per-tile sums of (count, occupied voxels) packed in 64 bits
//   k_scan_top            exclusive scan of the tile sums (one workgroup; on grids of at
//                         most FUSED_SCAN_TILES tiles k_scan_down adds them up itself)
//   k_scan_down           bin starts (exclusive prefix), occupied-voxel list, count reset
//   k_scatter      a4     cells into their bin's segment (arbitrary order inside it)
//   k_rank_gather  a4+a5  rank inside the bin by ascending id -> final slot; gather of the
//                         cell state into that order (+ the float and quantised shadows)
//   k_force_*      a6+a7  27-voxel neighbour forces -> velocity, Adams-Bashforth, walls;
//                         k_force_cells gives each XCD one contiguous run of cells
//   k_div_*               growing populations only: division after the walls
//   k_die_*               dying populations only: death after division
//   k_step_end            the bookkeeping alone, for a step without cells
// The paper measures the mechanics "update velocity" loop as the region that degrades
// when cells sit in memory in creation order rather than next to their neighbours in
// space (Section 5.4); here every step re-sorts cells by voxel, so the force kernel
// always reads neighbours that are contiguous in memory, and it visits only occupied
// voxels' cells (Section 5.4: skip empty voxels).  For the locality study the reorder
// can be skipped between steps (k_rank_perm instead of the gather; the force kernel then
// reads candidates through the sorted index), with bitwise the same results.
//
// Batches.  Every kernel serves a batch of independent simulations ("slots"): slot k
// owns the cell range [cell_off, cell_off + n_cells) and the voxel range
// [voxel_off, voxel_off + nx*ny*nz) of one arena, and its own domain and grid
// (SlotDesc).  Global voxel ids are voxel_off + the slot's own voxel id and global cell
// ids are cell_off + the slot's own cell id, so one global counting sort keeps every
// slot's cells inside its range and orders them exactly as the slot alone would be
// ordered: a simulation gives bitwise the same result alone and inside a batch.  The
// live sizes sit in a device header that the kernels read, so the captured step graph
// stays valid while slots are admitted and retired.  A single population is a batch of
// one slot.
//
// State layout (structure of arrays, one entry per cell, capacity-sized):
//   X[3]    f64  positions in storage order (integration output, binning input)
//   XS[3]   f64  positions gathered into this step's bin order (force input)
//   R[2]    f64  radius, T[2] i32 type, ID[2] u32 cell id, VP[2][3] v_prev (f64 or f32):
//                double-buffered; parity p holds them in the order of X
//   SH      float4 (x, y, z, r) in bin order, FP32 variants only
//   QS      8 bytes per cell in bin order: the quantised shadow the prefilter reads
//   slot_of u32  slot of the cell at each index (constant between repacks)
// Binning scratch: vid_cur, off, tmp_key, tmp_src, vid_sorted (u32 per cell);
// count, voxel_start (u32 per bin, XSUB bins per voxel), occ (u32 per voxel); tile sums
// (u64 per 2048 bins); the force kernel's work table (BAL_ENTRIES u32) and XCD split.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
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
constexpr uint32_t STAT_SLOTS = 1024;      // spread of the running counters
// Storage bins: each voxel is cut into XSUB slabs along x, and cells are stored bin by
// bin (voxel, then slab, then id).  A voxel is still one contiguous run (its XSUB bins),
// and the cells of a neighbour row that lie within reach of a cell along x are a
// contiguous run of whole slabs.
constexpr uint32_t XSUB = 4;
static_assert(SCAN_PER_THREAD % XSUB == 0 && SCAN_TILE % XSUB == 0, "scan tiles hold whole voxels");

// device header words
constexpr int H_CELLS = 0, H_VOXELS = 1, H_OCC = 2;
constexpr int H_STEP = 3;    // steps taken since creation (division draws)
constexpr int H_DIV = 4;     // cells that drew a division this step
constexpr int H_STEP_NOW = 5;  // the running step's index (H_STEP before it began)
constexpr int HDR_WORDS = 8;

// ------------------------------------------------------------------------ kernel args

// One simulation of a batch (device table, indexed by slot id).
// Device scratch of the allocation-free entry point (step_mechanics_noalloc): every
// array of its population is carved from here.  Each device the library runs on holds
// its own copy until the process ends.  Host code never uses this name as an address:
// it takes the device address from hipGetSymbolAddress (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[MECH_NOALLOC_SCRATCH_BYTES];

struct SlotDesc {
    double lo[3], hi[3];       // domain (reflecting walls), um
    double inv_h;              // 1 / voxel edge
    double r_max;              // largest radius of the slot's cells
    float r_max_f;
    int32_t nx, ny, nz;        // voxels per axis
    uint32_t voxel_off;        // first global voxel of the slot
    uint32_t cell_off;         // first cell index of the slot
    uint32_t prev_cell_off;    // cell_off before a repack (repack only)
    uint32_t n_cells;          // 0 marks a retired slot during a repack
    int32_t steps_left;        // > 0 steps to run, < 0 no limit, 0 frozen
    int32_t euler;             // the next step takes v_prev = v
    int32_t active_now;        // the running step advances the slot (steps_left was not 0)
    int32_t euler_now;         // the running step takes v_prev = v
    int32_t pad_[2];
    float q_scale;             // units per um of the quantised shadow: a power of two, h q_scale <= 2^13
    float q_pad;               // extra prefilter margin in units for float positions
};
static_assert(sizeof(SlotDesc) % 16 == 0, "SlotDesc alignment");

// Physics shared by the slots of a batch.
struct PhysArgs {
    double dt, c_rep, alpha, c_adh0;
    float c_rep_f, alpha_f, c_adh0_f, inv_alpha_f;   // inv_alpha_f = fl(1 / alpha_f)
    int32_t n_types, pad2_;
};

typedef unsigned short ushort2v __attribute__((ext_vector_type(2)));
typedef short short2v __attribute__((ext_vector_type(2)));
// margin of the prefilter's reach in units of the quantised shadow (3 > sqrt(3) + 1)
constexpr uint32_t Q_MARGIN = 3;
// entries of the quantised shadow past the last cell that the force kernel's trips may read
constexpr size_t QS_PAD = 16;
static_assert(QS_PAD >= 2 * 8, "a trip of up to 8 candidates from at most 7 past a row's end");

// The quantised shadow of a cell, the prefilter's input: each coordinate as
// round(x S) mod 2^16 (S = q_scale, a power of two, so x S is exact) and the reach
// ceil(alpha r S), packed (x | y << 16, z | reach << 16).  Differences of two cells of one
// 27-voxel neighbourhood are below 2 h S + 1 <= 2^14 + 1 units, so the 16-bit wrapped
// difference is the exact difference of the rounded coordinates.
// The float shadow (x, y, z, r) of a cell for the FP32 kernels.  Radii are positive, so
// with exactly two cell types the sign of r carries the type (negative for type 1): the
// two-type kernels then read no type per listed candidate.  Readers take |r|.
__device__ __forceinline__ float4 shadow(double x, double y, double z, double r, int32_t type, bool sign_type)
{
    const float w = (float)r;
    return make_float4((float)x, (float)y, (float)z, sign_type && type != 0 ? -w : w);
}

__device__ __forceinline__ float4 shadow_at(const float4* __restrict__ SH, uint32_t j)
{
    float4 v = SH[j];
    v.w = fabsf(v.w);
    return v;
}

__device__ __forceinline__ uint2 quantise(double x, double y, double z, double r, double S, double alpha)
{
    const uint32_t qx = (uint32_t)__double2ll_rn(x * S) & 0xffffu;
    const uint32_t qy = (uint32_t)__double2ll_rn(y * S) & 0xffffu;
    const uint32_t qz = (uint32_t)__double2ll_rn(z * S) & 0xffffu;
    const uint32_t qr = (uint32_t)ceil(alpha * r * S);
    return make_uint2(qx | (qy << 16), qz | (qr << 16));
}

// Candidates of one neighbour row a wave stages in LDS for its lanes (the union of their
// slab windows), and the padding a masked trip may read past them.
constexpr uint32_t STAGE_CAP = 256;
#ifndef MECH_STAGE_ROWS
#define MECH_STAGE_ROWS 1
#endif
constexpr bool STAGE_ROWS = MECH_STAGE_ROWS != 0;

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, WAVE));
    return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, WAVE));
    return v;
}

// Work table of the per-cell force kernel: BAL_ENTRIES sums of wave durations, each over
// `group` consecutive wave64s of cells (group grows with the population so the table
// covers it), read and cleared by one workgroup of the next step's k_bin.
constexpr uint32_t BAL_ENTRIES = 8192;
// the balanced runs are kept only when the uniform runs' fullest holds more than this
// share (in percent) above an even eighth of the measured work
constexpr uint32_t BAL_KEEP_PCT = 3;
__host__ __device__ inline uint32_t bal_group(uint32_t n)
{
    const uint32_t nw = (n + WAVE - 1) / WAVE;
    return nw > BAL_ENTRIES ? (nw + BAL_ENTRIES - 1) / BAL_ENTRIES : 1u;
}

// Workgroups are dealt to the 8 XCDs round robin; renumber the first nb of them so that
// each XCD gets a contiguous run of the voxel-ordered cells and its own L2 keeps the
// shared neighbours.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb)
{
    uint32_t xcd = b % N_XCD, k = b / N_XCD, q = nb / N_XCD, r = nb % N_XCD;
    return xcd < r ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

// a1: storage bin of a position in its slot's grid, XSUB * (voxel id) + x slab.
// (x - lo) * (1/h) is a subtraction then a product, so no fused form exists and the
// result is the IEEE value of the expression; multiplying it by XSUB (a power of two) is
// exact, so slab / XSUB is the voxel's x index floor((x - lo) * (1/h)), clamped alike.
__device__ __forceinline__ uint32_t bin_key(double x, double y, double z, const SlotDesc& d)
{
    double f0 = floor((x - d.lo[0]) * d.inv_h * (double)XSUB);
    double f1 = floor((y - d.lo[1]) * d.inv_h);
    double f2 = floor((z - d.lo[2]) * d.inv_h);
    f0 = fmin(fmax(f0, 0.0), (double)XSUB * (double)d.nx - 1.0);
    f1 = fmin(fmax(f1, 0.0), (double)(d.ny - 1));
    f2 = fmin(fmax(f2, 0.0), (double)(d.nz - 1));
    uint32_t k0 = (uint32_t)f0, k1 = (uint32_t)f1, k2 = (uint32_t)f2;
    return k0 + XSUB * (uint32_t)d.nx * (k1 + (uint32_t)d.ny * k2);
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

// Exclusive scan over a workgroup of NT threads (sh: NT / WAVE words); *total receives
// the workgroup sum.
template <int NT = BLOCK>
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t x, uint64_t* sh, uint64_t* total)
{
    uint64_t inc = wave_incl_scan(x);
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    if (lane == WAVE - 1) sh[w] = inc;
    __syncthreads();
    uint64_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / WAVE; ++i) {
        if (i < w) off += sh[i];
        tot += sh[i];
    }
    __syncthreads();
    *total = tot;
    return off + inc - x;
}

// Orders this wave's LDS accesses: writes by one lane are seen by the others after it.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------------ a1 + a2

// After the previous step's reorder the cells of one bin are adjacent, so the lanes of
// a wave fall into a few runs of equal bins and a per-lane atomic would hit the same
// counter many times over.  One lane per run adds the run's length; the run's lanes
// take consecutive offsets from the value it gets back.  Which cell of a bin gets which
// offset does not matter: a4 orders each bin's cells by id.  vid receives the global
// bin (XSUB * voxel_off + bin_key).
// The step's bookkeeping, done by the step's first kernel before any other reads it:
// whether each slot advances in this step and with which start of Adams-Bashforth, then
// its counters for the next step; and the step index.  (A step without cells runs
// k_step_end instead.)  `threads` threads starting at thread 0 of one workgroup.
__device__ __forceinline__ void begin_step(SlotDesc* slots, uint32_t n_slots, uint32_t* hdr, uint32_t tid,
                                           uint32_t threads)
{
    for (uint32_t t = tid; t < n_slots; t += threads) {
        SlotDesc& d = slots[t];
        const int32_t left = d.steps_left;
        d.active_now = left != 0 ? 1 : 0;
        d.euler_now = d.euler;
        if (left > 0) d.steps_left = left - 1;
        d.euler = 0;
    }
    if (tid == 0) {
        const uint32_t step = hdr[H_STEP];
        hdr[H_STEP_NOW] = step;
        hdr[H_STEP] = step + 1u;
    }
}

// The XCD runs of the next launch of k_force_cells, by one workgroup of BLOCK threads:
// cut the cells, in whole entries of the work table, into N_XCD runs of equal measured
// work (the wave durations the last launch added up) and clear the table.  The cut is
// kept when it beats the uniform runs (equal cell counts) by more than BAL_KEEP_PCT;
// split[N_XCD] = the cell count the cut was made for, or 0 for uniform runs.
__device__ __forceinline__ void balance_block(uint32_t* __restrict__ work, uint32_t n, uint32_t* __restrict__ split)
{
    constexpr uint32_t PER = BAL_ENTRIES / BLOCK;
    static_assert(PER % 4 == 0 && BAL_ENTRIES % BLOCK == 0, "each thread takes whole uint4s of the table");
    __shared__ unsigned long long s_wave[BLOCK / WAVE];
    __shared__ unsigned long long s_uni[N_XCD + 1];
    __shared__ uint32_t s_cut[N_XCD + 1];
    const uint32_t t = threadIdx.x, lane = t & (WAVE - 1);
    const uint4* const mine = reinterpret_cast<const uint4*>(work + t * PER);   // this thread's entries
    // the entries are loaded a few at a time where they are needed and not kept: this
    // block shares k_bin's register budget (62 VGPRs keep 8 waves per SIMD)
    unsigned long long own = 0;
#pragma unroll 4
    for (uint32_t k = 0; k < PER / 4; ++k) {
        const uint4 q = mine[k];
        own += (unsigned long long)q.x + q.y + q.z + q.w;
    }
    // block-wide inclusive scan of the threads' sums
    unsigned long long inc = own;
    for (int off = 1; off < WAVE; off <<= 1) {
        const unsigned long long v = __shfl_up(inc, off, WAVE);
        if (lane >= (uint32_t)off) inc += v;
    }
    if (lane == WAVE - 1) s_wave[t / WAVE] = inc;
    __syncthreads();
    unsigned long long total = 0;
    for (uint32_t i = 0; i < BLOCK / WAVE; ++i) {
        if (i < t / WAVE) inc += s_wave[i];
        total += s_wave[i];
    }
    const unsigned long long excl = inc - own;
    const bool cut = total >= (unsigned long long)N_XCD * N_XCD;   // else nothing measured: uniform runs
    const uint32_t group = bal_group(n);
#pragma unroll 1
    for (uint32_t q = 1; cut && q < N_XCD; ++q) {
        // the measured work before the uniform run q's first entry
        const uint32_t u = (uint32_t)(((uint64_t)n * q / N_XCD) / ((uint64_t)group * WAVE));
        // run q of the cut starts at the first entry whose preceding work reaches
        // q / N_XCD of the total
        const unsigned long long target = total * q / N_XCD;
        const bool uni = u / PER == t, at = excl < target && target <= inc;
        if (uni || at) {
            uint4 v[PER / 4];
#pragma unroll
            for (uint32_t k = 0; k < PER / 4; ++k) v[k] = mine[k];
            unsigned long long acc = excl, pre = excl;
            uint32_t end = PER;
#pragma unroll
            for (uint32_t j = 0; j < PER; ++j) {
                const uint32_t e = j % 4 == 0 ? v[j / 4].x : j % 4 == 1 ? v[j / 4].y : j % 4 == 2 ? v[j / 4].z : v[j / 4].w;
                if (j < u % PER) pre += e;
                if (acc < target) {
                    acc += e;
                    end = j + 1;
                }
            }
            if (uni) s_uni[q] = pre;
            if (at) s_cut[q] = t * PER + end;
        }
    }
    __syncthreads();   // every read of the table is done: clear it for the next launch
#pragma unroll 1
    for (uint32_t k = 0; k < PER / 4; ++k) reinterpret_cast<uint4*>(work + t * PER)[k] = make_uint4(0u, 0u, 0u, 0u);
    if (t == 0) {
        bool keep = false;
        if (cut) {
            s_uni[0] = 0;
            s_uni[N_XCD] = total;
            unsigned long long fullest = 0;
            for (uint32_t q = 0; q < N_XCD; ++q) fullest = max(fullest, s_uni[q + 1] - s_uni[q]);
            keep = fullest * 100u * N_XCD > total * (100u + BAL_KEEP_PCT);
        }
        if (keep) {
            split[0] = 0u;
            for (uint32_t q = 1; q < N_XCD; ++q)
                split[q] = (uint32_t)min<uint64_t>((uint64_t)s_cut[q] * group * WAVE, n);
        }
        split[N_XCD] = keep ? max(n, 1u) : 0u;
    }
}

__global__ __launch_bounds__(BLOCK) void k_bin(const double* __restrict__ px,
                                               const double* __restrict__ py,
                                               const double* __restrict__ pz,
                                               const uint32_t* __restrict__ slot_of,
                                               SlotDesc* __restrict__ slots,
                                               uint32_t* __restrict__ hdr,
                                               uint32_t* __restrict__ count,
                                               uint32_t* __restrict__ vid,
                                               uint32_t* __restrict__ off,
                                               uint32_t n_slots, int step_start,
                                               uint32_t* __restrict__ work, uint32_t* __restrict__ split)
{
    // with a work table, the grid's first workgroup (dispatched first, so it runs beside
    // the binning) cuts the force kernel's XCD runs; the others bin
    uint32_t bid = blockIdx.x, nbin = gridDim.x;
    if (work) {
        if (bid == 0) {
            balance_block(work, hdr[H_CELLS], split);
            return;
        }
        --bid;
        --nbin;
    }
    if (step_start && bid == 0) begin_step(slots, n_slots, hdr, threadIdx.x, BLOCK);
    const uint32_t n = hdr[H_CELLS];
    const uint32_t lane = threadIdx.x & (WAVE - 1);
    const uint64_t le = lane == WAVE - 1 ? ~0ull : (2ull << lane) - 1ull;  // lanes <= this one
    // the trip count is uniform per wave, so every lane takes part in the shuffles
    for (uint32_t s0 = bid * BLOCK + (threadIdx.x & ~(WAVE - 1)); s0 < n; s0 += nbin * BLOCK) {
        const uint32_t s = s0 + lane;
        const bool live = s < n;
        uint32_t v = 0xffffffffu;
        if (live) {
            const SlotDesc& d = slots[slot_of[s]];
            v = XSUB * d.voxel_off + bin_key(px[s], py[s], pz[s], d);
        }
        const uint32_t left = __shfl_up(v, 1, WAVE);
        const bool head = live && (lane == 0 || left != v);
        const uint64_t heads = __ballot(head);
        const uint64_t n_live = __popcll(__ballot(live));  // live lanes are a prefix
        const uint32_t first = 63u - (uint32_t)__clzll(heads & le);
        const uint64_t above = heads & ~le;
        const uint32_t end = above ? (uint32_t)__ffsll((long long)above) - 1u : (uint32_t)n_live;
        uint32_t base = 0;
        if (head) base = atomicAdd(&count[v], end - lane);
        base = __shfl(base, (int)first, WAVE);
        if (live) {
            off[s] = base + (lane - first);
            vid[s] = v;
        }
    }
}

// ------------------------------------------------------------------------ a3

// Scan words: low 32 bits count cells, high 32 bits count occupied voxels; both sums
// stay below 2^32.

// The scans run over the XSUB * V bins; the high word counts occupied voxels (a voxel
// is occupied when any of its bins is), flagged at the voxel's first bin.
__global__ __launch_bounds__(BLOCK) void k_scan_reduce(const uint32_t* __restrict__ count,
                                                       const uint32_t* __restrict__ hdr,
                                                       uint64_t* __restrict__ tsum)
{
    static_assert(XSUB == 4, "a voxel's bins are read as one uint4");
    __shared__ uint64_t sh[BLOCK / WAVE];
    const uint32_t V = hdr[H_VOXELS];
    const uint32_t S = XSUB * V;
    const uint32_t nt = (S + SCAN_TILE - 1) / SCAN_TILE;
    const uint4* count4 = reinterpret_cast<const uint4*>(count);   // one voxel per uint4
    for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
        const uint32_t base = tile * (SCAN_TILE / XSUB);
        uint64_t acc = 0;
#pragma unroll
        for (int k = 0; k < SCAN_PER_THREAD / XSUB; ++k) {
            const uint32_t v = base + k * BLOCK + threadIdx.x;
            if (v < V) {
                const uint4 q = count4[v];
                const uint32_t c = q.x + q.y + q.z + q.w;
                acc += (uint64_t)c | ((uint64_t)((q.x | q.y | q.z | q.w) != 0u) << 32);
            }
        }
        acc = wave_sum(acc);
        if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t t = 0;
            for (int i = 0; i < BLOCK / WAVE; ++i) t += sh[i];
            tsum[tile] = t;
        }
        __syncthreads();
    }
}

// One workgroup of TOP_BLOCK threads, in passes of TOP_CHUNK tile sums: a pass stages its
// sums in LDS with coalesced loads, each thread adds up a run of consecutive ones, and
// one workgroup scan per pass gives the prefixes, stored back coalesced.
constexpr int TOP_BLOCK = 1024;
constexpr uint32_t TOP_CHUNK = 8192;       // 64 KiB of LDS
constexpr uint32_t TOP_PER_THREAD = TOP_CHUNK / TOP_BLOCK;

__global__ __launch_bounds__(TOP_BLOCK) void k_scan_top(uint64_t* __restrict__ tsum,
                                                        uint32_t* __restrict__ voxel_start,
                                                        uint32_t* __restrict__ hdr)
{
    __shared__ uint64_t s_t[TOP_CHUNK];
    __shared__ uint64_t sh[TOP_BLOCK / WAVE];
    const uint32_t S = XSUB * hdr[H_VOXELS];
    const uint32_t nt = (S + SCAN_TILE - 1) / SCAN_TILE;
    const uint32_t b0 = threadIdx.x * TOP_PER_THREAD;
    uint64_t carry = 0;
    for (uint32_t base = 0; base < nt; base += TOP_CHUNK) {
        const uint32_t m = min(TOP_CHUNK, nt - base);
#pragma unroll
        for (uint32_t k = 0; k < TOP_PER_THREAD; ++k) {
            const uint32_t i = threadIdx.x + k * TOP_BLOCK;
            if (i < m) s_t[i] = tsum[base + i];
        }
        __syncthreads();
        uint64_t sum = 0;
#pragma unroll
        for (uint32_t k = 0; k < TOP_PER_THREAD; ++k)
            if (b0 + k < m) sum += s_t[b0 + k];
        uint64_t tot;
        uint64_t off = carry + block_excl_scan<TOP_BLOCK>(sum, sh, &tot);
#pragma unroll
        for (uint32_t k = 0; k < TOP_PER_THREAD; ++k) {
            if (b0 + k < m) {
                const uint64_t v = s_t[b0 + k];
                s_t[b0 + k] = off;
                off += v;
            }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t k = 0; k < TOP_PER_THREAD; ++k) {
            const uint32_t i = threadIdx.x + k * TOP_BLOCK;
            if (i < m) tsum[base + i] = s_t[i];
        }
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        voxel_start[S] = (uint32_t)carry;
        hdr[H_OCC] = (uint32_t)(carry >> 32);
    }
}

// FUSED (grids of at most FUSED_SCAN_TILES tiles): toff holds the raw tile sums and each
// workgroup adds up those before its tile itself, which saves the k_scan_top launch; the
// last tile's workgroup writes the totals.  Otherwise toff holds k_scan_top's exclusive
// prefix of the tile sums.
constexpr uint32_t FUSED_SCAN_TILES = 2048;

template <bool FUSED>
__global__ __launch_bounds__(BLOCK) void k_scan_down(uint32_t* __restrict__ count,
                                                     uint32_t* __restrict__ hdr,
                                                     const uint64_t* __restrict__ toff,
                                                     uint32_t* __restrict__ voxel_start,
                                                     uint32_t* __restrict__ occ)
{
    static_assert(SCAN_PER_THREAD == 8, "a thread's bins are read and written as two uint4");
    __shared__ __align__(16) uint32_t tile[SCAN_TILE];
    __shared__ uint64_t sh[BLOCK / WAVE];
    const uint32_t S = XSUB * hdr[H_VOXELS];
    const uint32_t nt = (S + SCAN_TILE - 1) / SCAN_TILE;
    if (FUSED && nt == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        voxel_start[0] = 0u;
        hdr[H_OCC] = 0u;
    }
    for (uint32_t ti = blockIdx.x; ti < nt; ti += gridDim.x) {
        const uint32_t base = ti * SCAN_TILE;
        uint64_t off0;
        if constexpr (FUSED) {
            uint64_t part = 0;
            for (uint32_t t = threadIdx.x; t < ti; t += BLOCK) part += toff[t];
            (void)block_excl_scan(part, sh, &off0);
        } else {
            off0 = toff[ti];
        }
#pragma unroll
        for (int k = 0; k < SCAN_PER_THREAD; ++k) {
            uint32_t v = base + k * BLOCK + threadIdx.x;
            tile[k * BLOCK + threadIdx.x] = v < S ? count[v] : 0u;
        }
        __syncthreads();
        // each thread holds whole voxels: bins t*SCAN_PER_THREAD + k
        uint32_t mine[SCAN_PER_THREAD];
        {
            const uint4 m0 = *reinterpret_cast<const uint4*>(tile + threadIdx.x * SCAN_PER_THREAD);
            const uint4 m1 = *reinterpret_cast<const uint4*>(tile + threadIdx.x * SCAN_PER_THREAD + 4);
            mine[0] = m0.x; mine[1] = m0.y; mine[2] = m0.z; mine[3] = m0.w;
            mine[4] = m1.x; mine[5] = m1.y; mine[6] = m1.z; mine[7] = m1.w;
        }
        uint64_t loc[SCAN_PER_THREAD];
        bool first_occ[SCAN_PER_THREAD];
        uint64_t sum = 0;
#pragma unroll
        for (int k = 0; k < SCAN_PER_THREAD; ++k) {
            bool f = false;
            if (k % XSUB == 0) {
                uint32_t any = 0;
#pragma unroll
                for (uint32_t m = 0; m < XSUB; ++m) any |= mine[k + m];
                f = any != 0u;
            }
            first_occ[k] = f;
            loc[k] = sum;
            sum += (uint64_t)mine[k] | ((uint64_t)f << 32);
        }
        uint64_t tot;
        uint64_t off = off0 + block_excl_scan(sum, sh, &tot);
        if constexpr (FUSED) {
            if (ti == nt - 1 && threadIdx.x == 0) {
                voxel_start[S] = (uint32_t)(off0 + tot);
                hdr[H_OCC] = (uint32_t)((off0 + tot) >> 32);
            }
        }
        const uint32_t v0 = base + threadIdx.x * SCAN_PER_THREAD;
        if (v0 + SCAN_PER_THREAD <= S) {
            // whole: two 16-byte stores (v0 is a multiple of 8 and the array 256-byte aligned)
            uint32_t ev[SCAN_PER_THREAD];
#pragma unroll
            for (int k = 0; k < SCAN_PER_THREAD; ++k) {
                const uint64_t e = off + loc[k];
                ev[k] = (uint32_t)e;
                if (first_occ[k]) occ[(uint32_t)(e >> 32)] = (v0 + k) / XSUB;
            }
            uint4* dst = reinterpret_cast<uint4*>(voxel_start + v0);
            dst[0] = make_uint4(ev[0], ev[1], ev[2], ev[3]);
            dst[1] = make_uint4(ev[4], ev[5], ev[6], ev[7]);
        } else {
#pragma unroll
            for (int k = 0; k < SCAN_PER_THREAD; ++k) {
                uint32_t v = v0 + k;
                if (v < S) {
                    uint64_t e = off + loc[k];
                    voxel_start[v] = (uint32_t)e;
                    if (first_occ[k]) occ[(uint32_t)(e >> 32)] = v / XSUB;
                }
            }
        }
        // the histogram of the next step starts from zero (empty bins already are: most
        // of a sparse grid's bins are not written at all)
#pragma unroll
        for (int k = 0; k < SCAN_PER_THREAD; ++k) {
            uint32_t v = base + k * BLOCK + threadIdx.x;
            if (v < S && tile[k * BLOCK + threadIdx.x] != 0u) count[v] = 0u;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------ a4 + a5

__global__ __launch_bounds__(BLOCK) void k_scatter(const uint32_t* __restrict__ hdr,
                                                   const uint32_t* __restrict__ vid,
                                                   const uint32_t* __restrict__ off,
                                                   const uint32_t* __restrict__ voxel_start,
                                                   const uint32_t* __restrict__ id_cur,
                                                   uint32_t* __restrict__ tmp_key,
                                                   uint32_t* __restrict__ tmp_src)
{
    const uint32_t n = hdr[H_CELLS];
    for (uint32_t s = blockIdx.x * BLOCK + threadIdx.x; s < n; s += gridDim.x * BLOCK) {
        uint32_t p = voxel_start[vid[s]] + off[s];
        tmp_key[p] = id_cur[s];
        tmp_src[p] = s;
    }
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
    double4* XR;             // FP64 records (x, y, z, r) of one-type arenas, or nullptr
    uint2* QS;               // quantised shadow (prefilter)
    int32_t sign_type;       // the shadow's sign carries the type (exactly two types)
    const uint32_t* slot_of;
    const SlotDesc* slots;
    double alpha;
    const uint32_t* vid_cur;
    const uint32_t* tmp_key;
    const uint32_t* tmp_src;
    const uint32_t* voxel_start;
    uint32_t* vid_sorted;
};

// Bins are short (a few to tens of cells), so each cell counts the smaller ids of its own
// bin directly; the cost is below that of the force loop over the same cells.
template <typename VPT>
__global__ __launch_bounds__(BLOCK) void k_rank_gather(const uint32_t* __restrict__ hdr, GatherArgs<VPT> a)
{
    const uint32_t n = hdr[H_CELLS];
    for (uint32_t p = blockIdx.x * BLOCK + threadIdx.x; p < n; p += gridDim.x * BLOCK) {
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
        const int32_t ty = a.T_cur[s];
        a.T_new[d] = ty;
        a.ID_new[d] = key;
#pragma unroll
        for (int c = 0; c < 3; ++c) a.VP_new[c][d] = a.VP_cur[c][s];
        a.vid_sorted[d] = v;
        if (a.SH) a.SH[d] = shadow(x, y, z, r, ty, a.sign_type != 0);
        if (a.XR) a.XR[d] = make_double4(x, y, z, r);
        a.QS[d] = quantise(x, y, z, r, (double)a.slots[a.slot_of[s]].q_scale, a.alpha);
    }
}

// ------------------------------------------------------------------------ a1..a5, small populations

// A population of at most SMALL_CELLS cells in at most SMALL_BINS bins is binned by one
// workgroup in one launch: counts, scan, scatter and the rank by id in LDS, then the
// gather.  Small populations are bound by launch latency, not bandwidth, and this
// replaces six dependent launches.  Same keys, scan, ranks and gather as the general
// path: the same order and outputs, bitwise.
constexpr uint32_t SMALL_CELLS = 8192;
constexpr uint32_t SMALL_BINS = 8192;
constexpr int SMALL_BLOCK = 1024;          // 16 waves: more loads in flight per phase
constexpr uint32_t SMALL_PER_THREAD = SMALL_CELLS / SMALL_BLOCK;
static_assert(SMALL_BINS / SMALL_BLOCK == SMALL_PER_THREAD && SMALL_PER_THREAD % XSUB == 0, "scan layout");

template <typename VPT>
__global__ __launch_bounds__(SMALL_BLOCK) void k_bin_small(const uint32_t* __restrict__ slot_of,
                                                     SlotDesc* __restrict__ slots,
                                                     uint32_t* __restrict__ hdr,
                                                     const uint32_t* __restrict__ id_cur,
                                                     uint32_t* __restrict__ vid_cur,
                                                     uint32_t* __restrict__ bin_start,
                                                     uint32_t* __restrict__ occ, GatherArgs<VPT> a,
                                                     uint32_t n_slots, int step_start)
{
    if (step_start) begin_step(slots, n_slots, hdr, threadIdx.x, SMALL_BLOCK);
    __shared__ uint32_t s_start[SMALL_BINS + 1];   // counts, then bin starts
    __shared__ uint32_t s_key[SMALL_CELLS];
    __shared__ uint32_t s_src[SMALL_CELLS];
    __shared__ uint32_t s_vid[SMALL_CELLS];
    __shared__ uint64_t sh[SMALL_BLOCK / WAVE];
    const uint32_t n = hdr[H_CELLS];
    const uint32_t S = XSUB * hdr[H_VOXELS];
    const uint32_t t = threadIdx.x;
    for (uint32_t b = t; b <= SMALL_BINS; b += SMALL_BLOCK) s_start[b] = 0u;
    __syncthreads();
    // a1 + a2
    uint32_t off[SMALL_PER_THREAD];
#pragma unroll
    for (uint32_t k = 0; k < SMALL_PER_THREAD; ++k) {
        const uint32_t s = t + k * SMALL_BLOCK;
        off[k] = 0;
        if (s < n) {
            const SlotDesc& d = slots[slot_of[s]];
            const uint32_t v = XSUB * d.voxel_off + bin_key(a.X[0][s], a.X[1][s], a.X[2][s], d);
            s_vid[s] = v;
            vid_cur[s] = v;
            off[k] = atomicAdd(&s_start[v], 1u);
        }
    }
    __syncthreads();
    // a3: each thread scans SMALL_PER_THREAD consecutive bins (whole voxels)
    const uint32_t b0 = t * SMALL_PER_THREAD;
    uint32_t cnt[SMALL_PER_THREAD];
    bool first_occ[SMALL_PER_THREAD];
    uint64_t loc[SMALL_PER_THREAD];
    uint64_t sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < SMALL_PER_THREAD; ++k) cnt[k] = b0 + k < S ? s_start[b0 + k] : 0u;
#pragma unroll
    for (uint32_t k = 0; k < SMALL_PER_THREAD; ++k) {
        bool f = false;
        if (k % XSUB == 0) {
            uint32_t any = 0;
#pragma unroll
            for (uint32_t m = 0; m < XSUB; ++m) any |= cnt[k + m];
            f = any != 0u;
        }
        first_occ[k] = f;
        loc[k] = sum;
        sum += (uint64_t)cnt[k] | ((uint64_t)f << 32);
    }
    uint64_t tot;
    const uint64_t base = block_excl_scan<SMALL_BLOCK>(sum, sh, &tot);   // synchronises the workgroup
#pragma unroll
    for (uint32_t k = 0; k < SMALL_PER_THREAD; ++k) {
        const uint32_t b = b0 + k;
        if (b < S) {
            const uint64_t e = base + loc[k];
            s_start[b] = (uint32_t)e;
            bin_start[b] = (uint32_t)e;
            if (first_occ[k]) occ[(uint32_t)(e >> 32)] = b / XSUB;
        }
    }
    if (t == 0) {
        s_start[S] = (uint32_t)tot;
        bin_start[S] = (uint32_t)tot;
        hdr[H_OCC] = (uint32_t)(tot >> 32);
    }
    __syncthreads();
    // a4: scatter into the bins, then rank by id
#pragma unroll
    for (uint32_t k = 0; k < SMALL_PER_THREAD; ++k) {
        const uint32_t s = t + k * SMALL_BLOCK;
        if (s < n) {
            const uint32_t p = s_start[s_vid[s]] + off[k];
            s_key[p] = id_cur[s];
            s_src[p] = s;
        }
    }
    __syncthreads();
    // a4 + a5: final slot and gather
    for (uint32_t p = t; p < n; p += SMALL_BLOCK) {
        const uint32_t s = s_src[p], key = s_key[p], v = s_vid[s];
        const uint32_t b = s_start[v], e = s_start[v + 1];
        uint32_t rank = 0;
        for (uint32_t q = b; q < e; ++q) rank += s_key[q] < key;
        const uint32_t d = b + rank;
        const double x = a.X[0][s], y = a.X[1][s], z = a.X[2][s];
        const double r = a.R_cur[s];
        a.XS[0][d] = x;
        a.XS[1][d] = y;
        a.XS[2][d] = z;
        a.R_new[d] = r;
        const int32_t ty = a.T_cur[s];
        a.T_new[d] = ty;
        a.ID_new[d] = key;
#pragma unroll
        for (int c = 0; c < 3; ++c) a.VP_new[c][d] = a.VP_cur[c][s];
        a.vid_sorted[d] = v;
        if (a.SH) a.SH[d] = shadow(x, y, z, r, ty, a.sign_type != 0);
        if (a.XR) a.XR[d] = make_double4(x, y, z, r);
        a.QS[d] = quantise(x, y, z, r, (double)a.slots[a.slot_of[s]].q_scale, a.alpha);
    }
}

// Cells left in place (the locality study): a4 only.  perm[slot] = storage index of the
// cell that the sorted order puts in that slot (the same (bin, id) order as a4 + a5).
__global__ __launch_bounds__(BLOCK) void k_rank_perm(const uint32_t* __restrict__ hdr,
                                                     const uint32_t* __restrict__ vid_cur,
                                                     const uint32_t* __restrict__ tmp_key,
                                                     const uint32_t* __restrict__ tmp_src,
                                                     const uint32_t* __restrict__ voxel_start,
                                                     uint32_t* __restrict__ perm)
{
    const uint32_t n = hdr[H_CELLS];
    for (uint32_t p = blockIdx.x * BLOCK + threadIdx.x; p < n; p += gridDim.x * BLOCK) {
        const uint32_t s = tmp_src[p];
        const uint32_t key = tmp_key[p];
        const uint32_t v = vid_cur[s];
        const uint32_t b = voxel_start[v], e = voxel_start[v + 1];
        uint32_t rank = 0;
        for (uint32_t q = b; q < e; ++q) rank += tmp_key[q] < key;
        perm[b + rank] = s;
    }
}

// Cells left in place: the new positions, written beside the old ones, become current.
__global__ __launch_bounds__(BLOCK) void k_commit(const uint32_t* __restrict__ hdr, const double* __restrict__ a0,
                                                  const double* __restrict__ a1, const double* __restrict__ a2,
                                                  double* __restrict__ b0, double* __restrict__ b1,
                                                  double* __restrict__ b2)
{
    const uint32_t n = hdr[H_CELLS];
    for (uint32_t s = blockIdx.x * BLOCK + threadIdx.x; s < n; s += gridDim.x * BLOCK) {
        b0[s] = a0[s];
        b1[s] = a1[s];
        b2[s] = a2[s];
    }
}

// Cells left in place: the float shadow and the FP64 records of the cells, in storage order.
__global__ __launch_bounds__(BLOCK) void k_shadow(const uint32_t* __restrict__ hdr, const double* __restrict__ x0,
                                                  const double* __restrict__ x1, const double* __restrict__ x2,
                                                  const double* __restrict__ r, float4* __restrict__ sh,
                                                  uint2* __restrict__ qs, const uint32_t* __restrict__ slot_of,
                                                  const SlotDesc* __restrict__ slots, double alpha,
                                                  const int32_t* __restrict__ type, int32_t sign_type,
                                                  double4* __restrict__ xr)
{
    const uint32_t n = hdr[H_CELLS];
    for (uint32_t s = blockIdx.x * BLOCK + threadIdx.x; s < n; s += gridDim.x * BLOCK) {
        if (sh) sh[s] = shadow(x0[s], x1[s], x2[s], r[s], sign_type != 0 ? type[s] : 0, sign_type != 0);
        if (xr) xr[s] = make_double4(x0[s], x1[s], x2[s], r[s]);
        qs[s] = quantise(x0[s], x1[s], x2[s], r[s], (double)slots[slot_of[s]].q_scale, alpha);
    }
}

// Before the cells are left in place: put them in id order (the order they were given
// in), with the state in the other buffer of each pair and the positions in XS.
template <typename VPT>
struct OrderArgs {
    const double* X[3];
    double* XS[3];
    const double* R_cur;
    double* R_new;
    const int32_t* T_cur;
    int32_t* T_new;
    const uint32_t* ID_cur;
    uint32_t* ID_new;
    const VPT* VP_cur[3];
    VPT* VP_new[3];
};

template <typename VPT>
__global__ __launch_bounds__(BLOCK) void k_order_by_id(const uint32_t* __restrict__ hdr, OrderArgs<VPT> a)
{
    const uint32_t n = hdr[H_CELLS];
    for (uint32_t p = blockIdx.x * BLOCK + threadIdx.x; p < n; p += gridDim.x * BLOCK) {
        const uint32_t d = a.ID_cur[p];  // global id: cell_off + index given at admission
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a.XS[c][d] = a.X[c][p];
            a.VP_new[c][d] = a.VP_cur[c][p];
        }
        a.R_new[d] = a.R_cur[p];
        a.T_new[d] = a.T_cur[p];
        a.ID_new[d] = d;
    }
}

// ------------------------------------------------------------------------ division

// Reflecting walls on a cell centre: mirror at each face, then clamp.
__device__ __forceinline__ double reflect(double x, double lo, double hi)
{
    if (x < lo) x = 2.0 * lo - x;
    if (x > hi) x = 2.0 * hi - x;
    return fmin(fmax(x, lo), hi);
}


// Growing populations: after the walls of step t, cell `id` divides when its first draw
// is below p_div.  Draws are counter-based: the SplitMix64 output function (Steele, Lea
// and Flood 2014) of the state seed + gamma * (4 (2^32 t + id) + k + 1), top 53 bits.
__device__ __forceinline__ double division_draw(uint64_t seed, uint32_t id, uint32_t t, uint32_t k)
{
    const uint64_t gamma = 0x9E3779B97F4A7C15ull;
    uint64_t z = seed + gamma * (4ull * (((uint64_t)t << 32) + id) + k + 1ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

struct DivArgs {
    double* X[3];
    double* R;
    int32_t* T;
    uint32_t* ID;
    void* VP[3];               // float or double, as the precision keeps v_prev
    uint32_t* slot_of;
    SlotDesc* slots;
    uint32_t* hdr;
    uint32_t* flag;            // indexed by id: 1 if the cell draws a division, then its rank
    uint64_t* tsum;            // tile sums of the rank scan
    uint64_t seed;
    double p_div;
    uint32_t capacity;         // cells the population may grow to
    uint32_t vp_bytes;         // 4 or 8
    // death: the probability, and the free buffers the survivors are gathered into
    double p_death;
    double* X_alt[3];
    double* R_alt;
    int32_t* T_alt;
    uint32_t* ID_alt;
    void* VP_alt[3];
};

__global__ __launch_bounds__(BLOCK) void k_div_mark(DivArgs a)
{
    const uint32_t n = a.hdr[H_CELLS], t = a.hdr[H_STEP_NOW];
    for (uint32_t s = blockIdx.x * BLOCK + threadIdx.x; s < n; s += gridDim.x * BLOCK) {
        const uint32_t id = a.ID[s];
        a.flag[id] = division_draw(a.seed, id, t, 0) < a.p_div ? 1u : 0u;
    }
}

// Exclusive scan of flag[0, n) by tiles: rank of each dividing cell among the dividing
// cells of smaller id.  The total goes to hdr[H_DIV].
__global__ __launch_bounds__(BLOCK) void k_div_scan_reduce(DivArgs a)
{
    __shared__ uint64_t sh[BLOCK / WAVE];
    const uint32_t n = a.hdr[H_CELLS];
    const uint32_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
    for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
        uint64_t acc = 0;
        for (int k = 0; k < SCAN_PER_THREAD; ++k) {
            const uint32_t v = tile * SCAN_TILE + k * BLOCK + threadIdx.x;
            if (v < n) acc += a.flag[v];
        }
        acc = wave_sum(acc);
        if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t tot = 0;
            for (int i = 0; i < BLOCK / WAVE; ++i) tot += sh[i];
            a.tsum[tile] = tot;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(BLOCK) void k_div_scan_top(DivArgs a)
{
    __shared__ uint64_t sh[BLOCK / WAVE];
    const uint32_t n = a.hdr[H_CELLS];
    const uint32_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
    uint64_t carry = 0;
    for (uint32_t base = 0; base < nt; base += BLOCK) {
        const uint32_t i = base + threadIdx.x;
        const uint64_t x = i < nt ? a.tsum[i] : 0;
        uint64_t tot;
        const uint64_t ex = block_excl_scan(x, sh, &tot);
        if (i < nt) a.tsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) a.hdr[H_DIV] = (uint32_t)carry;
}

__global__ __launch_bounds__(BLOCK) void k_div_scan_down(DivArgs a)
{
    __shared__ uint64_t sh[BLOCK / WAVE];
    const uint32_t n = a.hdr[H_CELLS];
    const uint32_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
    for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
        const uint32_t base = tile * SCAN_TILE + threadIdx.x * SCAN_PER_THREAD;
        uint32_t f[SCAN_PER_THREAD];
        uint64_t sum = 0;
        for (int k = 0; k < SCAN_PER_THREAD; ++k) {
            f[k] = base + k < n ? a.flag[base + k] : 0u;
            sum += f[k];
        }
        uint64_t tot;
        uint64_t off = a.tsum[tile] + block_excl_scan(sum, sh, &tot);
        for (int k = 0; k < SCAN_PER_THREAD; ++k) {
            if (base + k < n) a.flag[base + k] = (uint32_t)off;
            off += f[k];
        }
    }
}

// The dividing cells of rank below capacity - n divide: the daughter of rank k takes id
// and storage index n + k (appended at the end), the parent's radius, type and v_prev;
// parent and daughter move by -/+ r/2 along the drawn direction, through the walls.
__global__ __launch_bounds__(BLOCK) void k_div_apply(DivArgs a)
{
    const uint32_t n = a.hdr[H_CELLS], t = a.hdr[H_STEP_NOW];
    const uint32_t room = a.capacity - n;
    for (uint32_t s = blockIdx.x * BLOCK + threadIdx.x; s < n; s += gridDim.x * BLOCK) {
        const uint32_t id = a.ID[s];
        if (!(division_draw(a.seed, id, t, 0) < a.p_div)) continue;
        const uint32_t rank = a.flag[id];
        if (rank >= room) continue;
        double v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = 2.0 * division_draw(a.seed, id, t, (uint32_t)c + 1u) - 1.0;
        double e[3] = {0.0, 0.0, 1.0};
        {
#pragma clang fp contract(off)
            const double l2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            if (l2 >= 1e-12) {
                const double l = sqrt(l2);
#pragma unroll
                for (int c = 0; c < 3; ++c) e[c] = v[c] / l;
            }
        }
        const uint32_t q = n + rank;
        const SlotDesc& d = a.slots[a.slot_of[s]];
        const double half = 0.5 * a.R[s];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            {
#pragma clang fp contract(off)
                const double x = a.X[c][s];
                a.X[c][q] = reflect(x + half * e[c], d.lo[c], d.hi[c]);
                a.X[c][s] = reflect(x - half * e[c], d.lo[c], d.hi[c]);
            }
            if (a.vp_bytes == 4)
                static_cast<float*>(a.VP[c])[q] = static_cast<const float*>(a.VP[c])[s];
            else
                static_cast<double*>(a.VP[c])[q] = static_cast<const double*>(a.VP[c])[s];
        }
        a.R[q] = a.R[s];
        a.T[q] = a.T[s];
        a.ID[q] = n + rank;
        a.slot_of[q] = a.slot_of[s];
    }
}

__global__ void k_div_commit(DivArgs a)
{
    const uint32_t n = a.hdr[H_CELLS];
    const uint32_t room = a.capacity - n;
    const uint32_t grown = min(a.hdr[H_DIV], room);
    a.hdr[H_CELLS] = n + grown;
    a.slots[a.slot_of[0]].n_cells += grown;
}

// ------------------------------------------------------------------------ death

// Dying populations: after division in step t, cell `id` dies when its draw from the
// division generator with the seed's top bit flipped is below p_death (the two streams
// never share a state for t < 2^29).  The survivors keep their order by id and are
// renumbered 0, 1, ...: flag[id] = 1 for a survivor, scanned into its new id by the
// division scan kernels (the survivor count goes to hdr[H_DIV]); k_die_move gathers the
// survivors into the free buffers at their new ids, k_die_back copies them home, so the
// cells are stored in id order after the step.
__device__ __forceinline__ bool dies(const DivArgs& a, uint32_t id, uint32_t t)
{
    return division_draw(a.seed ^ 0x8000000000000000ull, id, t, 0) < a.p_death;
}

__global__ __launch_bounds__(BLOCK) void k_die_mark(DivArgs a)
{
    const uint32_t n = a.hdr[H_CELLS], t = a.hdr[H_STEP_NOW];
    for (uint32_t s = blockIdx.x * BLOCK + threadIdx.x; s < n; s += gridDim.x * BLOCK) {
        const uint32_t id = a.ID[s];
        a.flag[id] = dies(a, id, t) ? 0u : 1u;
    }
}

__global__ __launch_bounds__(BLOCK) void k_die_move(DivArgs a)
{
    const uint32_t n = a.hdr[H_CELLS], t = a.hdr[H_STEP_NOW];
    for (uint32_t s = blockIdx.x * BLOCK + threadIdx.x; s < n; s += gridDim.x * BLOCK) {
        const uint32_t id = a.ID[s];
        if (dies(a, id, t)) continue;
        const uint32_t d = a.flag[id];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a.X_alt[c][d] = a.X[c][s];
            if (a.vp_bytes == 4)
                static_cast<float*>(a.VP_alt[c])[d] = static_cast<const float*>(a.VP[c])[s];
            else
                static_cast<double*>(a.VP_alt[c])[d] = static_cast<const double*>(a.VP[c])[s];
        }
        a.R_alt[d] = a.R[s];
        a.T_alt[d] = a.T[s];
    }
}

__global__ __launch_bounds__(BLOCK) void k_die_back(DivArgs a)
{
    const uint32_t n = a.hdr[H_DIV];
    for (uint32_t d = blockIdx.x * BLOCK + threadIdx.x; d < n; d += gridDim.x * BLOCK) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a.X[c][d] = a.X_alt[c][d];
            if (a.vp_bytes == 4)
                static_cast<float*>(a.VP[c])[d] = static_cast<const float*>(a.VP_alt[c])[d];
            else
                static_cast<double*>(a.VP[c])[d] = static_cast<const double*>(a.VP_alt[c])[d];
        }
        a.R[d] = a.R_alt[d];
        a.T[d] = a.T_alt[d];
        a.ID[d] = d;
    }
}

__global__ void k_die_commit(DivArgs a)
{
    const uint32_t kept = a.hdr[H_DIV];
    a.slots[a.slot_of[0]].n_cells = kept;
    a.hdr[H_CELLS] = kept;
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

// ------------------------------------------------------------------------ a6 + a7 (shared)


template <typename VPT>
struct ForceArgs {
    const double* XS[3];
    const double* R;
    const int32_t* T;
    const float4* SH;
    const double4* XR;         // FP64 records (x, y, z, r) of one-type arenas, as XS and R; or nullptr
    const uint2* QS;
    const uint32_t* vid_sorted;
    const uint32_t* voxel_start;
    const uint32_t* slot_of;
    const SlotDesc* slots;
    const uint32_t* hdr;
    const double* cadh;        // n_types^2 (FP64)
    const float* cadh_f;       // n_types^2 (FP32)
    VPT* VP[3];                // read v_prev, write v (in place, own element)
    double* X[3];              // new positions
    const uint32_t* perm;      // cells left in place: storage index of each sorted slot
    unsigned long long* stats; // STAT_SLOTS pairs (interactions, candidates)
    uint32_t* work;            // BAL_ENTRIES sums of wave durations, zero before the launch (or null)
    const uint32_t* split;     // first cell of each XCD's run, from the durations (or null)
};

// a7 for one cell: two-step Adams-Bashforth from the gathered position, reflecting
// walls of its slot, history <- v.
// x0: the gathered position when the caller holds it, else null (read from XS).
template <typename VPT>
__device__ __forceinline__ void integrate(const ForceArgs<VPT>& a, const PhysArgs& P, const SlotDesc& d,
                                          uint32_t i, const double v[3], const double* x0 = nullptr)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double vp = d.euler_now ? v[c] : (double)a.VP[c][i];
        const double xn = (x0 ? x0[c] : a.XS[c][i]) + P.dt * (1.5 * v[c] - 0.5 * vp);
        a.X[c][i] = reflect(xn, d.lo[c], d.hi[c]);
        a.VP[c][i] = (VPT)v[c];
    }
}

// A frozen slot (its steps are done) keeps its state: the gathered position is copied
// back and the gathered history is left as it is.
template <typename VPT>
__device__ __forceinline__ void hold(const ForceArgs<VPT>& a, uint32_t i, const double* x0 = nullptr)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) a.X[c][i] = x0 ? x0[c] : a.XS[c][i];
}

// 1/sqrt(x) and 1/x in FP64 from the hardware estimates (about 24 correct bits) and one
// Newton step each: measured on gfx950 within 19.5 ulp (rsqrt), 36 ulp (x * rsqrt(x) as
// sqrt) and 11 ulp (reciprocal) of the exact values over 2^-12 .. 2^12.  They replace
// the correctly rounded square root and three divisions of the pair term; the in-range
// decision is on d2 and is unchanged.  A second step each (within 1.8, 2.2 and 0.5 ulp)
// made the FP64 force kernel 2% slower and the results no closer to the FP64 oracle.
__device__ __forceinline__ double rsqrt_nr(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    return y * fma(-h * y, y, 1.5);
}

__device__ __forceinline__ double rcp_nr(double x)
{
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}

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
        // both comparisons as one predicate (not short-circuit): one branch per pair
        if (!((d2 > 0.0) & (d2 < RA * RA))) return false;
    }
    const double inv_d = rsqrt_nr(d2);
    const double d = d2 * inv_d;
    double w = 0.0;
    if (d < R) {
        double u = 1.0 - d * rcp_nr(R);
        w = c_rep * u * u;
    }
    double a = 1.0 - d * rcp_nr(RA);
    w -= cadh * a * a;
    double s = w * inv_d;
    ax += s * dx;
    ay += s * dy;
    az += s * dz;
    return true;
}

// FP32 pair term on the float shadow.  The decision is the IEEE float result of the
// written expressions, each operation rounded on its own (d2 = (dx*dx + dy*dy) + dz*dz,
// R and R_A rounded to float; no fused forms).  1/d from the hardware reciprocal square
// root, 1/R from the hardware reciprocal, and 1/R_A as (1/R) fl(1/alpha): one
// transcendental fewer per pair than 1/R_A of its own.  With KAHAN the three sums are
// Kahan-compensated (Kahan 1965): cmp carries the low part the last addition lost and is
// taken off the next term; the running sum is the result.
template <bool KAHAN>
__device__ __forceinline__ bool pair32(float xi, float yi, float zi, float ri, float4 q,
                                       float alpha, float c_rep, float cadh, float* acc,
                                       float* cmp, float inv_alpha)
{
    float dx, dy, dz, d2, R, RA;
    {
#pragma clang fp contract(off)
        dx = xi - q.x;
        dy = yi - q.y;
        dz = zi - q.z;
        d2 = dx * dx + dy * dy + dz * dz;
        R = ri + q.w;
        RA = alpha * R;
        if (!((d2 > 0.0f) & (d2 < RA * RA))) return false;
    }
    float inv_d = __builtin_amdgcn_rsqf(d2);
    float d = d2 * inv_d;
    const float inv_R = __builtin_amdgcn_rcpf(R);
    float w = 0.0f;
    if (d < R) {
        float u = 1.0f - d * inv_R;
        w = c_rep * u * u;
    }
    float a = 1.0f - d * (inv_R * inv_alpha);
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

// In-range decision only, with the same expressions, uncontracted, as pair64 / pair32.
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
    const float d2 = dx * dx + dy * dy + dz * dz;
    const float RA = alpha * (me.w + c.w);
    return d2 > 0.0f && d2 < RA * RA;
}

// Running counters are spread over STAT_SLOTS pairs (summed when read): device-scope
// atomics on one address from every wave of the GPU serialise at the memory side.
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

// Neighbour geometry of a cell: its voxel coordinates in its slot and the x-range of
// the three voxels of each neighbour row.
struct Cellgeo {
    int kx, ky, kz, x0, x1;
};

__device__ __forceinline__ Cellgeo cell_geo(uint32_t gvox, const SlotDesc& d)
{
    Cellgeo g;
    const uint32_t v = gvox - d.voxel_off;
    g.kx = (int)(v % (uint32_t)d.nx);
    g.ky = (int)((v / (uint32_t)d.nx) % (uint32_t)d.ny);
    g.kz = (int)(v / ((uint32_t)d.nx * (uint32_t)d.ny));
    g.x0 = g.kx > 0 ? g.kx - 1 : 0;
    g.x1 = g.kx < d.nx - 1 ? g.kx + 1 : d.nx - 1;
    return g;
}

// Global voxel id of the first voxel of neighbour row q (dz = q/3 - 1, dy = q%3 - 1),
// or -1 when the row lies outside the slot's grid.
__device__ __forceinline__ int64_t row_first(const Cellgeo& g, const SlotDesc& d, int q)
{
    const int y = g.ky + (q % 3) - 1, z = g.kz + (q / 3) - 1;
    if (y < 0 || y >= d.ny || z < 0 || z >= d.nz) return -1;
    return (int64_t)d.voxel_off + (int64_t)d.nx * ((int64_t)y + (int64_t)d.ny * z) + g.x0;
}

// ------------------------------------------------------------------------ a6 + a7, row kernel

// One thread per cell in storage (bin) order.  The 27 neighbour voxels are visited as 9
// rows (dz, dy); the three voxels of a row (dx = -1, 0, 1) are adjacent in the sorted
// order, so a row is one contiguous range of the sorted arrays, read in the oracle's
// order.  Every candidate of the 27 voxels is tested (no slab window).
// PREC: 0 FP64, 1 FP32, 2 FP32 + Kahan.  MULTI: more than one cell type.
template <int PREC, bool MULTI, typename VPT>
__device__ __forceinline__ void force_rows_cell(const PhysArgs& P, const ForceArgs<VPT>& a, uint32_t i,
                                                uint32_t& inter, uint32_t& cand)
{
    {
        const SlotDesc& d = a.slots[a.slot_of[i]];
        if (!d.active_now) {
            hold(a, i);
        } else {
            const Cellgeo g = cell_geo(a.vid_sorted[i] / XSUB, d);
            const int ti = MULTI ? a.T[i] : 0;
            double v[3];
            if (PREC == 0) {
                const double xi = a.XS[0][i], yi = a.XS[1][i], zi = a.XS[2][i];
                const double ri = a.R[i];
                double ax = 0.0, ay = 0.0, az = 0.0;
                for (int q = 0; q < 9; ++q) {
                    const int64_t r0 = row_first(g, d, q);
                    if (r0 < 0) continue;
                    const uint32_t b = a.voxel_start[XSUB * r0];
                    const uint32_t e = a.voxel_start[XSUB * (r0 + (g.x1 - g.x0) + 1)];
                    cand += e - b;
                    for (uint32_t j = b; j < e; ++j) {
                        const double c = MULTI ? a.cadh[ti * P.n_types + a.T[j]] : P.c_adh0;
                        inter += pair64(xi, yi, zi, ri, a.XS[0][j], a.XS[1][j], a.XS[2][j],
                                        a.R[j], P.alpha, P.c_rep, c, ax, ay, az);
                    }
                }
                v[0] = ax;
                v[1] = ay;
                v[2] = az;
            } else {
                const float4 me = shadow_at(a.SH, i);
                float acc[3] = {0.f, 0.f, 0.f}, cmp[3] = {0.f, 0.f, 0.f};
                for (int q = 0; q < 9; ++q) {
                    const int64_t r0 = row_first(g, d, q);
                    if (r0 < 0) continue;
                    const uint32_t b = a.voxel_start[XSUB * r0];
                    const uint32_t e = a.voxel_start[XSUB * (r0 + (g.x1 - g.x0) + 1)];
                    cand += e - b;
                    for (uint32_t j = b; j < e; ++j) {
                        const float c = MULTI ? a.cadh_f[ti * P.n_types + a.T[j]] : P.c_adh0_f;
                        inter += pair32<PREC == 2>(me.x, me.y, me.z, me.w, shadow_at(a.SH, j), P.alpha_f,
                                                   P.c_rep_f, c, acc, cmp, P.inv_alpha_f);
                    }
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c] = (double)acc[c];
            }
            cand -= 1;  // the cell itself
            integrate(a, P, d, i, v);
        }
    }
}

// The cells of the batch in blocks of WPB wave64s, taken in rounds of gridDim.x blocks;
// in each round the active blocks are renumbered so that each XCD gets a contiguous run.
template <int PREC, bool MULTI, typename VPT, int WPB>
__global__ __launch_bounds__(WPB * WAVE) void k_force_rows(PhysArgs P, ForceArgs<VPT> a)
{
    constexpr uint32_t TB = WPB * WAVE;
    const uint32_t n = a.hdr[H_CELLS];
    const uint32_t nb = (n + TB - 1) / TB;
    uint32_t inter = 0, cand = 0;
    for (uint32_t lb0 = 0; lb0 < nb; lb0 += gridDim.x) {
        const uint32_t active = min(gridDim.x, nb - lb0);
        if (blockIdx.x >= active) break;
        const uint32_t i = (lb0 + xcd_block(blockIdx.x, active)) * TB + threadIdx.x;
        if (i < n) force_rows_cell<PREC, MULTI, VPT>(P, a, i, inter, cand);
    }
    add_stats(a.stats, inter, cand);
}

// ------------------------------------------------------------------------ a6 + a7, list kernel

// LIST: candidates a lane can hold listed before a flush (16, 32 or 64).
// UNROLL: candidates tested per loop trip (independent loads in flight), at most LIST / 2.

// One thread per cell in storage (bin) order.  Each lane walks its 9 neighbour rows,
// reading in each only the x slabs within reach of its cell (a contiguous run: slabs of
// x-adjacent voxels follow each other), and only prefilters the candidates, FC_UNROLL
// loads in flight per trip.  The prefilter runs on the quantised shadow (8 bytes per
// cell: the coordinates in units of 1/S um wrapped to 16 bits, and the reach
// ceil(alpha r S)) in every precision, in exact integer arithmetic: a candidate is
// listed in LDS when its squared distance in units is below (reach_i + reach_j)^2, the
// lane's reach carrying a margin that covers the rounding of the coordinates and of the
// exact decision (see `near`).  Half the bytes of the float shadow per candidate, and a
// 16-bit packed difference and an int16 dot product in place of float arithmetic.
// When a list fills, and at the end,
// the lanes evaluate their listed candidates together with the exact decision and
// pair term of pair64 / pair32, in candidate order, so each sum is still taken in the
// fixed neighbour order and the rare interacting pairs do not make the wave diverge.
// Lanes of one slab read the same candidate at the same time (one cache line).
// IND: the cells are left in storage order; candidate slot j of the sorted order is read
// through perm[j] (the locality study).  The candidates, their order and the arithmetic
// are those of the reordered path, so the results are bitwise the same.
// PRUNE: the per-cell pruned walk (below) instead of the slab window walk.
template <int PREC, bool MULTI, typename VPT, int FC_UNROLL, int LIST, bool IND = false, bool PRUNE = false>
__device__ __forceinline__ void force_cells_cell(const PhysArgs& P, const ForceArgs<VPT>& a, uint32_t i,
                                                 uint32_t n, uint32_t* const list0, uint2* const rng0,
                                                 uint2* const stage0, const void* const cadh_lds,
                                                 uint32_t& inter, uint32_t& cand)
{
    // the slab walk stages shared rows in LDS (stage0: STAGE_CAP + FC_UNROLL entries); in
    // the one-type FP64 kernel only, whose candidate stream limits it most (the others ran
    // slower with the registers staging takes)
    constexpr bool STAGE = !PRUNE && !IND && PREC == 0 && !MULTI && STAGE_ROWS;
    // one-type FP64: the cell's own position and radius come from its record as well,
    // so the kernel reads neither XS nor R
    constexpr bool REC = PREC == 0 && !MULTI;
    using Real = typename std::conditional<PREC == 0, double, float>::type;
    const bool in_pop = i < n;
    const uint32_t ii = in_pop ? i : n - 1;  // idle lanes mirror the last cell
    double4 rec{};
    if constexpr (REC) rec = a.XR[ii];
    const double r_own = REC ? rec.w : a.R[ii];
    const SlotDesc& d = a.slots[a.slot_of[ii]];
    const bool valid = in_pop && d.active_now != 0;
    const Cellgeo g = cell_geo(a.vid_sorted[ii] / XSUB, d);
    // Slab window (default walk): the x slabs of each neighbour row that can hold a
    // partner: every interacting j has |x_j - x_i| < alpha (r_i + r_max).  The window is
    // taken in FP64 from the exact position and widened by a margin that covers the
    // float rounding of the FP32 decision (a few ulp of |x|) and of R_A, so it never drops
    // a pair either precision counts.  w0, w1: the window's first and one-past-last slab,
    // counted from the first slab of the row's voxels and clipped to them.
    uint32_t w0 = 0, w1 = 0;
    if constexpr (!PRUNE) {
        const double xg = REC ? rec.x : a.XS[0][ii];
        const double reach = P.alpha * (r_own + d.r_max);
        const double m = reach * (1.0 + 1e-6) + 1e-3 + 5e-7 * (fabs(xg) + reach);
        const double xs = (double)XSUB * d.inv_h;
        const double lo_s = floor((xg - d.lo[0] - m) * xs), hi_s = floor((xg - d.lo[0] + m) * xs);
        const double s_min = (double)(XSUB * (uint32_t)g.x0), s_max = (double)(XSUB * (uint32_t)g.x1 + XSUB - 1);
        w0 = (uint32_t)(fmax(lo_s, s_min) - s_min);            // first slab, from the row's start
        w1 = (uint32_t)(fmin(hi_s, s_max) - s_min) + 1u;       // one past the last slab
    }
    // Pruned walk: the candidates of each neighbour row that can hold a partner, the
    // paper's test of
    // whether a neighbour voxel can hold interacting cells (Section 4.2) done per cell and
    // row: every interacting j has d_ij < reach = alpha (r_i + r_max), so with rho the
    // distance in y-z from the cell to the row's voxels, a row with rho >= reach holds no
    // partner and is skipped, and in the others |x_j - x_i| < sqrt(reach^2 - rho^2): the
    // row's x slabs in that window are one contiguous run of the sorted arrays.  The reach
    // is taken in FP64 from the exact position and widened by a margin that covers the
    // float rounding of the FP32 decision (a few ulp of |x|) and of R_A; the window
    // arithmetic then runs in float on coordinates in voxel units relative to the cell's
    // own voxel (exact to about 1e-7 of a voxel), under a further relative pad of 1e-5.
    // So a window never drops a pair that either precision counts.  The non-empty runs,
    // in row order (dz, then dy), go to the lane's LDS slots rng0[k * WAVE], k < nr.
    uint32_t nr = 0;
    if (PRUNE && valid) {
        const double xg = REC ? rec.x : a.XS[0][ii], yg = REC ? rec.y : a.XS[1][ii], zg = REC ? rec.z : a.XS[2][ii];
        const double reach = P.alpha * (r_own + d.r_max);
        const double pm = fmax(fabs(xg), fmax(fabs(yg), fabs(zg)));
        const double m = reach * (1.0 + 1e-6) + 1e-3 + 5e-7 * (pm + reach);
        const float rh = (float)(m * d.inv_h) * (1.0f + 1e-5f);           // voxel units
        const float rh2 = rh * rh;
        const float uy = (float)((yg - d.lo[1]) * d.inv_h - (double)g.ky);  // in [0, 1]
        const float uz = (float)((zg - d.lo[2]) * d.inv_h - (double)g.kz);
        // x in slabs from the first slab of the row's voxels, and the row's last slab
        const float sx = (float)(((xg - d.lo[0]) * d.inv_h - (double)g.x0) * (double)XSUB);
        const float s_last = (float)(XSUB * (uint32_t)(g.x1 - g.x0 + 1) - 1u);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int dz = q / 3 - 1, dy = q % 3 - 1;
            // distance from the cell to the row's voxels along y and z, in voxel units
            const float ey = fmaxf(dy < 0 ? uy : dy > 0 ? 1.0f - uy : 0.0f, 0.0f);
            const float ez = fmaxf(dz < 0 ? uz : dz > 0 ? 1.0f - uz : 0.0f, 0.0f);
            const float t = rh2 - (ey * ey + ez * ez);
            const int64_t r0 = row_first(g, d, q);
            if (r0 >= 0 && t > 0.0f) {
                const float hw = __builtin_sqrtf(t) * (float)XSUB;
                const uint32_t w0 = (uint32_t)fmaxf(floorf(sx - hw), 0.0f);
                const uint32_t w1 = (uint32_t)fminf(floorf(sx + hw), s_last) + 1u;
                if (w1 > w0) {
                    const uint32_t jb = a.voxel_start[XSUB * r0 + w0];
                    const uint32_t je = a.voxel_start[XSUB * r0 + w1];
                    if (je > jb) {
                        rng0[nr * WAVE] = make_uint2(jb, je);
                        ++nr;
                        cand += je - jb;
                    }
                }
            }
        }
    }
    Real xi, yi, zi, ri;
    if constexpr (REC) {
        xi = rec.x;
        yi = rec.y;
        zi = rec.z;
        ri = rec.w;
    } else if constexpr (PREC == 0) {
        xi = a.XS[0][ii];
        yi = a.XS[1][ii];
        zi = a.XS[2][ii];
        ri = a.R[ii];
    } else {
        const float4 m = shadow_at(a.SH, ii);
        xi = m.x;
        yi = m.y;
        zi = m.z;
        ri = m.w;
    }
    // the prefilter's lane constants: the quantised (x | y << 16) and (z | 0) of the cell,
    // and its reach ceil(alpha r_i S) plus the margin (below)
    const uint2 qi = a.QS[ii];
    const uint32_t q_xy = qi.x, q_z = qi.y & 0xffffu;
    const uint32_t q_a = (uint32_t)ceil(P.alpha * r_own * (double)d.q_scale) + Q_MARGIN + (uint32_t)d.q_pad;
    const int ti = MULTI ? a.T[ii] : 0;
    Real acc[3] = {0, 0, 0}, cmp[3] = {0, 0, 0};
    // The short list (LIST = 16, picked for dense populations) is a ring,
    // list0[(k mod LIST) * WAVE]: the listed entries run from head up to tail
    // (excluded), oldest first, and a flush inside the walk evaluates only the oldest
    // entries (below).  In the ring an entry is up to EB candidates of a trip:
    // (j << EB) | m, the candidates j + u with bit u of m set (j < 2^(32 - EB); EB = 8 for
    // trips of 8 of one cell type, else 4), so a trip of EB writes one entry.  The
    // long lists (32, 64: small populations, few waves per SIMD) and the walk through
    // perm hold one candidate per entry, from list0, emptied whole.  Every trip writes
    // its entry at tail, which advances only when the entry holds a candidate (no
    // branch).  The ring stays below LIST - EPT entries before a trip and the lists below
    // LIST - FC_UNROLL, so a list never holds more than LIST - 1 and, in the ring,
    // (tail - head) mod LIST is its exact length.
    constexpr bool RING = LIST < 32;
    constexpr bool PACK = RING && !IND;
    constexpr uint32_t MASK = RING ? (uint32_t)LIST - 1u : 0xffffffffu;
    static_assert(!RING || (LIST & (LIST - 1)) == 0, "the ring length is a power of two");
    // candidates per packed entry, packed entries a trip writes, entries after which a
    // trip flushes, and entries a lane may keep after a flush: the packed ring flushes
    // only as much as the next trip needs, so that each pass finds entries in as many
    // lanes as possible (measured: 2% faster than keeping 10 of 16)
    // (entries of 8 for trips of 8 of one cell type: the single-type tumour ran 7% faster
    // in FP32 with them, the two-type batch of spheroids 4% slower)
    constexpr uint32_t EB = FC_UNROLL == 8 && !MULTI ? 8u : 4u, EMASK = (1u << EB) - 1u;
    constexpr uint32_t EPT = ((uint32_t)FC_UNROLL + EB - 1u) / EB;
    constexpr uint32_t FULL = PACK ? (uint32_t)LIST - EPT : (uint32_t)(LIST - FC_UNROLL);
    constexpr uint32_t KEEP = PACK ? FULL - 1u : RING ? (uint32_t)LIST * 5u / 8u : 0u;
    static_assert(KEEP < FULL, "a flush makes room for the next trip");
    uint32_t head = 0, tail = 0, done = 0;  // done: bits of the head entry already evaluated
    auto push = [&](uint32_t e, bool in) {
        list0[tail * WAVE] = e;
        tail = (tail + (in ? 1u : 0u)) & MASK;
    };
    auto count = [&]() { return (tail - head) & MASK; };
    auto full = [&]() { return __any(count() >= FULL); };

    // The prefilter on a candidate's quantised shadow c: with D the squared distance of
    // the rounded coordinates in units (exact: 16-bit wrapped differences, an int16
    // dot product) and t = q_a + ceil(alpha r_j S), the candidate is listed when D < t^2.
    // Each rounded difference is within 1 unit of (x_i - x_j) S, so sqrt(D) is within
    // sqrt(3) of d S; an interacting pair has d < alpha (r_i + r_j) up to the relative
    // rounding of its decision (2^-50 in FP64, a few 2^-24 in FP32, there plus the
    // rounding of the positions to float, at most 2^-22 P S units, which q_pad covers),
    // so sqrt(D) < t - Q_MARGIN + 2 and every interacting pair is listed.
    // The test takes D - t^2 in int32 from three int16 pairs: du = (dx, dy), w = (dz, -t)
    // and (dz, t), with D - t^2 = du.du + w.(dz, t).  t < 2^15 (each reach is at most 2^12
    // units and the domain check bounds q_pad), so -t is an int16; |D - t^2| < 2^31.  The
    // sign bit of D - t^2 is the decision.
    const uint32_t q_zt = q_z | ((0u - q_a) & 0xffffu) << 16;   // (q_z, -q_a) as two int16
    auto gap = [&](uint2 c) -> int {
        const short2v du = __builtin_bit_cast(
            short2v, __builtin_bit_cast(ushort2v, q_xy) - __builtin_bit_cast(ushort2v, c.x));
        const short2v w = __builtin_bit_cast(
            short2v, __builtin_bit_cast(ushort2v, q_zt) - __builtin_bit_cast(ushort2v, c.y));
        const short2v wt = w * (short2v){1, -1};
        // clamp set on the first product (it never saturates: |dz^2 - t^2| < 2^31) selects the
        // three-operand form, whose zero addend is an inline constant and not a register move
        return __builtin_amdgcn_sdot2(du, du, __builtin_amdgcn_sdot2(w, wt, 0, true), false);
    };
    auto near = [&](uint2 c) -> bool { return gap(c) < 0; };
    // bit u set when candidate c[u] is listed, u < N: the signs shifted in from the last
    auto bits = [&](const uint2* c, auto N) -> uint32_t {
        uint32_t m = 0;
#pragma unroll
        for (int u = decltype(N)::value - 1; u >= 0; --u) m = __builtin_amdgcn_alignbit(m, (uint32_t)gap(c[u]), 31);
        return m;
    };
    // The candidate data a flush evaluates.  With the long lists (few waves per SIMD
    // hide little latency) the next entry's data is fetched before the current one is
    // evaluated; with the short list the extra registers would cost a wave per SIMD,
    // which matters more.
    struct Cand {
        Real x, y, z, r;
        int t;
    };
    auto fetch = [&](uint32_t j) {
        Cand c;
        if constexpr (PREC == 0) {
            if constexpr (!MULTI) {
                // one 32-byte record instead of four gathers
                const double4 v = a.XR[j];
                c.x = v.x;
                c.y = v.y;
                c.z = v.z;
                c.r = v.w;
            } else {
                c.x = a.XS[0][j];
                c.y = a.XS[1][j];
                c.z = a.XS[2][j];
                c.r = a.R[j];
            }
            c.t = MULTI ? a.T[j] : 0;
        } else {
            const float4 v = a.SH[j];
            c.x = v.x;
            c.y = v.y;
            c.z = v.z;
            c.r = fabsf(v.w);
            // with exactly two types the shadow's sign is the type: no type load
            c.t = MULTI ? (P.n_types == 2 ? (v.w < 0.0f ? 1 : 0) : a.T[j]) : 0;
        }
        return c;
    };
    auto eval = [&](const Cand& c) {
        if constexpr (PREC == 0) {
            const double cadh = MULTI ? static_cast<const double*>(cadh_lds)[ti * P.n_types + c.t] : P.c_adh0;
            inter += pair64(xi, yi, zi, ri, c.x, c.y, c.z, c.r, P.alpha, P.c_rep, cadh, acc[0], acc[1], acc[2]);
        } else {
            const float cadh = MULTI ? static_cast<const float*>(cadh_lds)[ti * P.n_types + c.t] : P.c_adh0_f;
            inter += pair32<PREC == 2>(xi, yi, zi, ri, make_float4(c.x, c.y, c.z, c.r), P.alpha_f, P.c_rep_f,
                                       cadh, acc, cmp, P.inv_alpha_f);
        }
    };
    // The ring evaluates in every lane the candidates of its oldest entries, one per pass
    // and in candidate order, until the fullest list is down to `keep` entries (all of
    // them when keep is 0).  Each pass keeps every lane that still holds an entry busy,
    // where emptying whole lists would leave the lanes with short lists idle for most of
    // the passes.  A long list is emptied whole, the next entry's data fetched before
    // the current one is evaluated.
    auto flush = [&](uint32_t keep) {
        if constexpr (PACK) {
#pragma unroll 1
            for (;;) {
                const uint32_t c = count();
                if (!__any(c > keep)) break;
                if (c > 0) {
                    const uint32_t e = list0[head * WAVE];
                    const uint32_t m = e & EMASK & ~done;
                    const uint32_t b = (uint32_t)__builtin_ctz(m);
                    eval(fetch((e >> EB) + b));
                    const bool last = (m & (m - 1u)) == 0u;
                    done = last ? 0u : done | (1u << b);
                    head = (head + (last ? 1u : 0u)) & MASK;
                }
            }
        } else if constexpr (!RING) {
            const uint32_t c = count();
            Cand cn = fetch(c > 0 ? list0[0] : ii);
#pragma unroll 1
            for (uint32_t k = 0; k < (uint32_t)LIST; ++k) {
                if (!__any(k < c)) break;
                const Cand cur = cn;
                // entries at and above c are stale: the own cell stands in for them
                cn = fetch(k + 1 < c ? list0[(k + 1) * WAVE] : ii);
                if (k < c) eval(cur);
            }
            tail = 0;
        } else {
            const uint32_t c = count();
            uint32_t k = 0;
#pragma unroll 1
            for (; k < (uint32_t)LIST; ++k) {
                if (!__any(k + keep < c)) break;
                if (k < c) eval(fetch(list0[((head + k) & MASK) * WAVE]));
            }
            head = (head + min(c, k)) & MASK;
        }
    };

    if constexpr (!PRUNE) {
        // The slab walk: the lanes take the 9 rows together; in each, a lane reads its
        // window's candidates FC_UNROLL per trip (lanes of one slab read the same
        // candidate at the same time, one cache line).  The candidate range [j, e) of
        // neighbour row q (empty outside the grid); the next row's range is read while
        // the current row is walked.
        auto range = [&](int q, uint32_t& j, uint32_t& e) {
            const int64_t r0 = valid ? row_first(g, d, q) : -1;
            j = r0 < 0 ? 0u : a.voxel_start[XSUB * r0 + w0];
            e = r0 < 0 ? 0u : a.voxel_start[XSUB * r0 + w1];
        };
        if constexpr (STAGE) {
            // A row's candidates [j, e) from src (src[0] is candidate j): trips of FC_UNROLL,
            // then one masked trip for the rest.
            auto walk = [&](auto sp, uint32_t j, const uint32_t e) {
                for (; j + FC_UNROLL <= e; j += FC_UNROLL, sp += FC_UNROLL) {
                    uint2 c[FC_UNROLL];
    #pragma unroll
                    for (int u = 0; u < FC_UNROLL; ++u) c[u] = sp[u];
                    if constexpr (PACK) {
                        const uint32_t mb = bits(c, std::integral_constant<int, FC_UNROLL>{});
                        if constexpr (EB == 8) {
                            push((j << 8) | mb, mb != 0u);
                        } else {
    #pragma unroll
                            for (int g4 = 0; g4 < FC_UNROLL; g4 += 4) {
                                const uint32_t m = (mb >> g4) & 15u;
                                push(((j + g4) << 4) | m, m != 0u);
                            }
                        }
                    } else {
    #pragma unroll
                        for (int u = 0; u < FC_UNROLL; ++u) push(j + u, near(c[u]));
                    }
                    if (full()) flush(KEEP);
                }
                // fewer than FC_UNROLL left: one more trip, testing only the candidates below e
                // (the shadow array is padded by QS_PAD >= 2 FC_UNROLL entries past the last
                // cell and the stage by FC_UNROLL, so a trip that starts below e reads inside
                // them; a lane with nothing left reads from its e and lists nothing)
                if (__any(j < e)) {
                    const uint32_t lim = j < e ? e - j : 0u;
                    uint2 c[FC_UNROLL];
    #pragma unroll
                    for (int u = 0; u < FC_UNROLL; ++u) c[u] = sp[u];
                    if constexpr (PACK) {
                        // the bits at and past the row's end are masked off (lim < FC_UNROLL)
                        const uint32_t mb = bits(c, std::integral_constant<int, FC_UNROLL>{}) & ((1u << lim) - 1u);
                        if constexpr (EB == 8) {
                            push((j << 8) | mb, mb != 0u);
                        } else {
    #pragma unroll
                            for (int g4 = 0; g4 < FC_UNROLL; g4 += 4) {
                                const uint32_t m = (mb >> g4) & 15u;
                                push(((j + g4) << 4) | m, m != 0u);
                            }
                        }
                    } else {
    #pragma unroll
                        for (int u = 0; u < FC_UNROLL; ++u) push(j + u, near(c[u]) & ((uint32_t)u < lim));
                    }
                    if (full()) flush(KEEP);
                }
            };
            // Shared rows: when the wave's working lanes sit in one y-z row of voxels of one
            // simulation (the common case: 64 consecutive cells span two or three voxels along
            // x), they read the same 9 neighbour rows, and each lane's slab window is one
            // range [A0, A1) of absolute x slabs, the same in every row.  The wave then stages
            // the union of the lanes' windows of a row, [U0, U1), into LDS once (coalesced,
            // one load per candidate instead of one per lane that reads it) and the lanes walk
            // their own windows there: the vector memory return path carried each lane's copy.
            // Rows whose union exceeds the stage, and waves that span two rows, walk from the
            // shadow in memory.  Same candidates, same order: the results are unchanged.
            bool share = false;
            uint32_t s_min = 0, s_max = 0, s_base = 0;
            int s_ky = 0, s_kz = 0, s_nx = 0, s_ny = 0, s_nz = 0;
            if constexpr (STAGE) {
                const uint64_t vm = __ballot(valid);
                if (vm != 0u) {
                    const int ref = __ffsll((long long)vm) - 1;
                    s_ky = __shfl(g.ky, ref, WAVE);
                    s_kz = __shfl(g.kz, ref, WAVE);
                    const uint32_t voff = (uint32_t)__shfl((int)d.voxel_off, ref, WAVE);
                    share = __all(!valid || (g.ky == s_ky && g.kz == s_kz && d.voxel_off == voff));
                    if (share) {
                        // every row decision below uses the working lanes' simulation (lanes of a
                        // finished one, or idle lanes, may hold another): wave-uniform values
                        const uint32_t a0 = (uint32_t)(XSUB * g.x0) + w0, a1 = (uint32_t)(XSUB * g.x0) + w1;
                        s_min = __builtin_amdgcn_readfirstlane(wave_min_u32(valid ? a0 : 0xffffffffu));
                        s_max = __builtin_amdgcn_readfirstlane(wave_max_u32(valid ? a1 : 0u));
                        s_ky = __builtin_amdgcn_readfirstlane(s_ky);
                        s_kz = __builtin_amdgcn_readfirstlane(s_kz);
                        s_base = __builtin_amdgcn_readfirstlane(voff);
                        s_nx = __builtin_amdgcn_readfirstlane(__shfl(d.nx, ref, WAVE));
                        s_ny = __builtin_amdgcn_readfirstlane(__shfl(d.ny, ref, WAVE));
                        s_nz = __builtin_amdgcn_readfirstlane(__shfl(d.nz, ref, WAVE));
                    }
                }
            }
            uint32_t j_next, e_next;
            range(0, j_next, e_next);
            for (int q = 0; q < 9; ++q) {
                uint32_t j = j_next;
                const uint32_t e = e_next;
                if (q < 8) range(q + 1, j_next, e_next);
                cand += e - j;
                if constexpr (IND) {
                    // gathers through the sorted order: no locality between consecutive lanes
                    for (; j < e; ++j) {
                        const uint32_t jj = a.perm[j];
                        push(jj, near(a.QS[jj]));
                        if (full()) flush(KEEP);
                    }
                    continue;
                }
                if constexpr (STAGE) {
                    if (share) {
                        const int y = s_ky + q % 3 - 1, z = s_kz + q / 3 - 1;
                        if (y < 0 || y >= s_ny || z < 0 || z >= s_nz) continue;   // no row: every window empty
                        const uint32_t b = XSUB * (s_base + (uint32_t)s_nx * ((uint32_t)y + (uint32_t)s_ny * (uint32_t)z));
                        const uint32_t u0 = a.voxel_start[b + s_min], u1 = a.voxel_start[b + s_max];
                        if (u1 - u0 <= STAGE_CAP) {
                            __builtin_amdgcn_wave_barrier();   // the last row's reads are issued
                            for (uint32_t k = threadIdx.x & (WAVE - 1); k < u1 - u0; k += WAVE) stage0[k] = a.QS[u0 + k];
                            __builtin_amdgcn_wave_barrier();   // ... and this row's writes, before its reads
                            // a lane with no window (idle, or its simulation done) has j = e = 0:
                            // its masked trip reads from the stage's start
                            walk(stage0 + (j >= u0 ? j - u0 : 0u), j, e);
                            continue;
                        }
                    }
                }
                walk(a.QS + j, j, e);
            }
        } else {
            uint32_t j_next, e_next;
            range(0, j_next, e_next);
            for (int q = 0; q < 9; ++q) {
                uint32_t j = j_next;
                const uint32_t e = e_next;
                if (q < 8) range(q + 1, j_next, e_next);
                cand += e - j;
                if constexpr (IND) {
                    // gathers through the sorted order: no locality between consecutive lanes
                    for (; j < e; ++j) {
                        const uint32_t jj = a.perm[j];
                        push(jj, near(a.QS[jj]));
                        if (full()) flush(KEEP);
                    }
                    continue;
                }
                const uint2* sp = a.QS + j;
                for (; j + FC_UNROLL <= e; j += FC_UNROLL, sp += FC_UNROLL) {
                    uint2 c[FC_UNROLL];
    #pragma unroll
                    for (int u = 0; u < FC_UNROLL; ++u) c[u] = sp[u];
                    if constexpr (PACK) {
                        const uint32_t mb = bits(c, std::integral_constant<int, FC_UNROLL>{});
                        if constexpr (EB == 8) {
                            push((j << 8) | mb, mb != 0u);
                        } else {
    #pragma unroll
                            for (int g4 = 0; g4 < FC_UNROLL; g4 += 4) {
                                const uint32_t m = (mb >> g4) & 15u;
                                push(((j + g4) << 4) | m, m != 0u);
                            }
                        }
                    } else {
    #pragma unroll
                        for (int u = 0; u < FC_UNROLL; ++u) push(j + u, near(c[u]));
                    }
                    if (full()) flush(KEEP);
                }
                // fewer than FC_UNROLL left: one more trip, testing only the candidates below e
                // (the shadow array is padded by QS_PAD >= 2 FC_UNROLL entries past the last
                // cell, so a trip that starts below e reads inside it; a lane with nothing left
                // reads from its e and lists nothing)
                if (__any(j < e)) {
                    const uint32_t lim = j < e ? e - j : 0u;
                    uint2 c[FC_UNROLL];
    #pragma unroll
                    for (int u = 0; u < FC_UNROLL; ++u) c[u] = sp[u];
                    if constexpr (PACK) {
                        // the bits at and past the row's end are masked off (lim < FC_UNROLL)
                        const uint32_t mb = bits(c, std::integral_constant<int, FC_UNROLL>{}) & ((1u << lim) - 1u);
                        if constexpr (EB == 8) {
                            push((j << 8) | mb, mb != 0u);
                        } else {
    #pragma unroll
                            for (int g4 = 0; g4 < FC_UNROLL; g4 += 4) {
                                const uint32_t m = (mb >> g4) & 15u;
                                push(((j + g4) << 4) | m, m != 0u);
                            }
                        }
                    } else {
    #pragma unroll
                        for (int u = 0; u < FC_UNROLL; ++u) push(j + u, near(c[u]) & ((uint32_t)u < lim));
                    }
                    if (full()) flush(KEEP);
                }
            }
        }
    } else {
        // The walk: each lane takes its own runs one after the other, FC_UNROLL candidates
        // per trip, so a trip of the wave serves every lane that still has candidates,
        // whichever row it is in (lanes of one wave sit in two or three voxels and at
        // different depths of them, so their runs differ in number and length).  A trip reads
        // FC_UNROLL consecutive entries of the quantised shadow from j; those at or past the
        // run's end e are not listed (the array is padded, so the reads stay inside it, and a
        // lane that has finished re-reads from its last e).  When j passes e the lane moves
        // to its next run.  Candidates are listed in run order, so each sum is still taken in
        // the fixed neighbour order.
        uint32_t k = 0;
        uint2 run = nr > 0 ? rng0[0] : make_uint2(0u, 0u);
        uint32_t j = run.x, e = run.y;
    #pragma unroll 1
        while (__any(k < nr)) {
            const uint32_t lim = k < nr ? min(e - j, (uint32_t)FC_UNROLL) : 0u;
            if constexpr (IND) {
                // gathers through the sorted order: no locality between consecutive lanes
    #pragma unroll
                for (int u = 0; u < FC_UNROLL; ++u) {
                    uint32_t jj = ii;
                    bool in = false;
                    if ((uint32_t)u < lim) {
                        jj = a.perm[j + u];
                        in = near(a.QS[jj]);
                    }
                    push(jj, in);
                }
            } else {
                uint2 c[FC_UNROLL];
    #pragma unroll
                for (int u = 0; u < FC_UNROLL; ++u) c[u] = a.QS[j + u];
                if constexpr (PACK) {
                    const uint32_t mb = bits(c, std::integral_constant<int, FC_UNROLL>{}) & ((1u << lim) - 1u);
                    if constexpr (EB == 8) {
                        push((j << 8) | mb, mb != 0u);
                    } else {
    #pragma unroll
                        for (int g4 = 0; g4 < FC_UNROLL; g4 += 4) {
                            const uint32_t m = (mb >> g4) & 15u;
                            push(((j + g4) << 4) | m, m != 0u);
                        }
                    }
                } else {
    #pragma unroll
                    for (int u = 0; u < FC_UNROLL; ++u) push(j + u, (uint32_t)u < lim && near(c[u]));
                }
            }
            j += FC_UNROLL;
            if (k < nr && j >= e) {
                ++k;
                run = k < nr ? rng0[k * WAVE] : make_uint2(e, e);
                j = run.x;
                e = run.y;
            }
            if (full()) flush(KEEP);
        }
    }
    flush(0);
    if (valid) {
        cand -= 1;  // the cell itself
        double v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = (double)acc[c];
        if constexpr (REC) {
            const double x0[3] = {rec.x, rec.y, rec.z};
            integrate(a, P, d, i, v, x0);
        } else {
            integrate(a, P, d, i, v);
        }
    } else if (in_pop) {
        if constexpr (REC) {
            const double x0[3] = {rec.x, rec.y, rec.z};
            hold(a, i, x0);
        } else {
            hold(a, i);
        }
    }
}

// Waves per SIMD the register allocation of a force kernel is asked to fit (1: as
// compiled), measured per shape on the tumour and the batch:
// * the staged one-type FP64 ring kernels, 6 (80 VGPRs, none spilled in the default
//   shape; the compiler would take 88 and hold 5): 3% faster;
// * the one-wave FP32 kernels with trips of 8 and 16-entry rings, 8 (64 VGPRs): the
//   two-type batch kernel fits without spills (71 as compiled, 7 waves) and ran 4%
//   faster, the one-type FP32 + Kahan kernel spills two (73, 6 waves) and ran 1% faster;
// * the two-type FP64 kernels held at 6 instead of 5 were 4% slower, the one-type FP32
//   kernel held at 8 (70 VGPRs as compiled) 0.6% slower, and the one-type FP32 + Kahan
//   kernel held at 7 no faster: those stay as compiled.
template <int PREC, bool MULTI, int WPB, int UNROLL, int LIST, bool IND, bool PRUNE>
constexpr int force_waves_per_simd()
{
    if (IND || PRUNE || LIST != 16) return 1;
    if (PREC == 0) return !MULTI && STAGE_ROWS ? 6 : 1;
    return WPB == 1 && UNROLL == 8 && (MULTI ? PREC == 1 : PREC == 2) ? 8 : 1;
}

template <int PREC, bool MULTI, typename VPT, int WPB, int UNROLL, int LIST, bool IND = false, bool PRUNE = false>
__global__ __launch_bounds__(WPB * WAVE)
__attribute__((amdgpu_waves_per_eu(force_waves_per_simd<PREC, MULTI, WPB, UNROLL, LIST, IND, PRUNE>())))
void k_force_cells(PhysArgs P, ForceArgs<VPT> a)
{
    static_assert(2 * UNROLL <= LIST, "a trip must fit the list above the flush mark");
    constexpr uint32_t TB = WPB * WAVE;
    __shared__ uint32_t s_list[WPB][LIST][WAVE];
    const uint32_t n = a.hdr[H_CELLS];
    const uint32_t nb = (n + TB - 1) / TB;
    uint32_t* const list0 = &s_list[threadIdx.x / WAVE][0][threadIdx.x & (WAVE - 1)];
    uint2* rng0 = nullptr;
    uint2* stage0 = nullptr;
    if constexpr (PRUNE) {
        // the pruned walk's runs
        __shared__ uint2 s_rng[WPB][9][WAVE];
        rng0 = &s_rng[threadIdx.x / WAVE][0][threadIdx.x & (WAVE - 1)];
    } else if constexpr (!IND && PREC == 0 && !MULTI && STAGE_ROWS) {
        // the slab walk's staged row
        __shared__ uint2 s_stage[WPB][STAGE_CAP + UNROLL];
        stage0 = &s_stage[threadIdx.x / WAVE][0];
    }
    const void* cadh_lds = nullptr;
    if constexpr (MULTI) {
        // The adhesion table (n_types^2 <= 64 entries) in LDS, read once per listed
        // candidate: read from global memory it took the load return path that bounds
        // the two-type kernels (the batch ran 6% slower, the 100k spheroid 5%).
        using Real = typename std::conditional<PREC == 0, double, float>::type;
        __shared__ Real s_cadh[WPB][64];
        Real* const tab = &s_cadh[threadIdx.x / WAVE][0];
        const uint32_t l = threadIdx.x & (WAVE - 1);
        if (l < (uint32_t)(P.n_types * P.n_types)) {
            if constexpr (PREC == 0) tab[l] = a.cadh[l];
            else tab[l] = a.cadh_f[l];
        }
        __builtin_amdgcn_wave_barrier();   // the wave's writes before its reads
        cadh_lds = tab;
    }
    uint32_t inter = 0, cand = 0;
    // Each XCD takes one contiguous run of tiles, so its L2 keeps the neighbours its
    // cells share; the runs hold equal shares of the last launch's measured work, or
    // equal numbers of tiles before there is any.  The runs partition [0, nb) whatever
    // the split holds: the bounds are clamped and made non-decreasing.
    const uint32_t X = min(gridDim.x, N_XCD);
    const uint32_t x = blockIdx.x % X, nbx = (gridDim.x - x + X - 1) / X;
    uint32_t t0, t1;
    if (a.split && X == N_XCD && a.split[N_XCD] != 0u) {
        uint32_t lo = 0, hi = 0;
#pragma unroll
        for (uint32_t q = 1; q <= N_XCD; ++q) {
            const uint32_t b = q == N_XCD ? nb : max(hi, min((a.split[q] + TB / 2) / TB, nb));
            if (q == x) lo = b;
            hi = b;
            if (q == x + 1) break;
        }
        t0 = x == 0 ? 0u : lo;
        t1 = hi;
    } else {
        // equal runs, the longer ones on the XCDs that the round robin gives one
        // workgroup more: with a tile per workgroup, no workgroup takes two
        const uint32_t q = nb / X, r = nb % X;
        t0 = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
        t1 = t0 + q + (x < r ? 1u : 0u);
    }
    const uint32_t group = bal_group(n);
    for (uint32_t t = t0 + blockIdx.x / X; t < t1; t += nbx) {
        // read unconditionally: a conditional read costs the FP64 kernels a register
        const uint64_t c0 = wall_clock64();
        force_cells_cell<PREC, MULTI, VPT, UNROLL, LIST, IND, PRUNE>(P, a, t * TB + threadIdx.x, n, list0, rng0,
                                                                     stage0, cadh_lds, inter, cand);
        if (a.work) {
            // the wave's index among the wave64s of cells; waves past the last cell record
            // nothing, so the entry (wave / group) is below BAL_ENTRIES
            const uint32_t wave = t * WPB + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
            if ((threadIdx.x & (WAVE - 1)) == 0 && wave * WAVE < n)
                atomicAdd(&a.work[wave / group], (uint32_t)max<uint64_t>(wall_clock64() - c0, 1));
        }
    }
    add_stats(a.stats, inter, cand);
}

// ------------------------------------------------------------------------ a6 + a7, voxel kernel

// Per-wave LDS: the candidates of one chunk of the 27-voxel neighbourhood (x, y, z, r),
// their types, and per-lane lists of in-range candidate indices.
constexpr int FL_WAVES = 4;                // waves per workgroup
constexpr int FL_LIST = 16;                // list entries per lane before a flush

template <int PREC> struct Stage;
template <> struct Stage<0> { using T = double4; static constexpr int CAP = 256; };
template <> struct Stage<1> { using T = float4; static constexpr int CAP = 512; };
template <> struct Stage<2> { using T = float4; static constexpr int CAP = 512; };

// One wave per occupied voxel: the waves of the grid walk the non-empty voxel list with
// a fixed stride (empty voxels cost nothing).  The wave stages its 27-voxel
// neighbourhood in LDS (9 rows, each a contiguous range of the voxel-ordered arrays)
// and splits its lanes as (target, slice): target t of r = min(64, remaining) takes
// lanes t, t + r, ..., so all 64 lanes test candidates.  A lane appends the in-range
// candidates of its slice to an LDS list and evaluates them in a batch, so the force
// arithmetic does not diverge on the rare in-range branch.  Slices are combined in a
// fixed order: results are bitwise reproducible.
template <int PREC, bool MULTI, typename VPT>
__global__ __launch_bounds__(FL_WAVES * WAVE) void k_force_lds(PhysArgs P, ForceArgs<VPT> a,
                                                               const uint32_t* __restrict__ occ)
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
    const uint32_t M = a.hdr[H_OCC];
    uint32_t inter = 0, cand = 0;

    // wave q of the (XCD-renumbered) grid takes occupied voxels q, q + W, q + 2W, ...
    const uint32_t nwaves = gridDim.x * FL_WAVES;
    const uint32_t q0 = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * FL_WAVES + w);
    for (uint32_t o = q0; o < M; o += nwaves) {
        const uint32_t vox = __builtin_amdgcn_readfirstlane(occ[o]);
        const uint32_t vb = a.voxel_start[XSUB * vox], k = a.voxel_start[XSUB * vox + XSUB] - vb;
        const SlotDesc& d = a.slots[__builtin_amdgcn_readfirstlane(a.slot_of[vb])];
        if (!d.active_now) {
            for (uint32_t t = lane; t < k; t += WAVE) hold(a, vb + t);
            continue;
        }
        const Cellgeo g = cell_geo(vox, d);
        // the 9 rows in (dz, dy) order; rows outside the grid are empty
        uint32_t rb[9], pre[10];
        pre[0] = 0;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int64_t r0 = row_first(g, d, q);
            uint32_t b = 0, e = 0;
            if (r0 >= 0) {
                b = a.voxel_start[XSUB * r0];
                e = a.voxel_start[XSUB * (r0 + (g.x1 - g.x0) + 1)];
            }
            rb[q] = b;
            pre[q + 1] = pre[q] + (e - b);
        }
        const uint32_t C = pre[9];

        for (uint32_t t0 = 0; t0 < k; t0 += WAVE) {
            const uint32_t r = min((uint32_t)WAVE, k - t0);
            const uint32_t t = (uint32_t)lane % r, s = (uint32_t)lane / r;
            const uint32_t St = (uint32_t)WAVE / r + (t < (uint32_t)WAVE % r ? 1u : 0u);
            const uint32_t i = vb + t0 + t;
            CT me;
            if constexpr (PREC == 0) {
                me = make_double4(a.XS[0][i], a.XS[1][i], a.XS[2][i], a.R[i]);
            } else {
                me = shadow_at(a.SH, i);
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
                            pair32<PREC == 2>(me.x, me.y, me.z, me.w, c, P.alpha_f, P.c_rep_f, cadh, acc, cmp,
                                              P.inv_alpha_f);
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
                    uint32_t gi = ff + rb[0];
#pragma unroll
                    for (int q = 1; q < 9; ++q)
                        if (ff >= pre[q]) gi = ff - pre[q] + rb[q];
                    if constexpr (PREC == 0) {
                        stage[f] = make_double4(a.XS[0][gi], a.XS[1][gi], a.XS[2][gi], a.R[gi]);
                    } else {
                        stage[f] = shadow_at(a.SH, gi);
                    }
                    if (MULTI) s_type[w][f] = (uint8_t)a.T[gi];
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
            // combine the slices' sums of each target in slice order
            wave_sync();
            Real* part = reinterpret_cast<Real*>(stage);
#pragma unroll
            for (int c = 0; c < 3; ++c) part[lane * 3 + c] = acc[c];
            wave_sync();
            if (s == 0) {
                Real tot[3] = {0, 0, 0}, tc[3] = {0, 0, 0};
                for (uint32_t q = 0; q < St; ++q) {
                    const uint32_t l = t + q * r;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const Real term = part[l * 3 + c];
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
                double v[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c] = (double)tot[c];
                integrate(a, P, d, i, v);
            }
            wave_sync();
        }
    }
    add_stats(a.stats, inter, cand);
}

// ------------------------------------------------------------------------ step end, slots

// Counts down the steps of every slot still running; a slot that reaches 0 is frozen
// from the next step on.  The first step has been taken, so no slot starts with Euler.
__global__ __launch_bounds__(BLOCK) void k_step_end(SlotDesc* __restrict__ slots, uint32_t n_slots,
                                                    uint32_t* __restrict__ hdr)
{
    const uint32_t t = blockIdx.x * BLOCK + threadIdx.x;
    if (t == 0) hdr[H_STEP] += 1u;
    if (t >= n_slots) return;
    if (slots[t].steps_left > 0) slots[t].steps_left -= 1;
    slots[t].euler = 0;
}

__global__ void k_set_slot(SlotDesc* __restrict__ slots, uint32_t id, SlotDesc d) { slots[id] = d; }

__global__ void k_set_header(uint32_t* __restrict__ hdr, uint32_t n_cells, uint32_t n_voxels)
{
    hdr[H_CELLS] = n_cells;
    hdr[H_VOXELS] = n_voxels;
}

// Moves the cells of the live slots to their new offsets (the slot table holds the old
// and new offsets; n_cells == 0 marks a retired slot, whose cells are dropped).
template <typename VPT>
struct RepackArgs {
    const double* X[3];
    double* XS[3];
    const double* R_cur;
    double* R_new;
    const int32_t* T_cur;
    int32_t* T_new;
    const uint32_t* ID_cur;
    uint32_t* ID_new;
    const VPT* VP_cur[3];
    VPT* VP_new[3];
    const uint32_t* slot_of;
    uint32_t* slot_new;
    const SlotDesc* slots;
};

template <typename VPT>
__global__ __launch_bounds__(BLOCK) void k_repack(uint32_t n_old, RepackArgs<VPT> a)
{
    const uint32_t s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= n_old) return;
    const uint32_t k = a.slot_of[s];
    const SlotDesc& d = a.slots[k];
    if (d.n_cells == 0) return;
    const uint32_t t = d.cell_off + (s - d.prev_cell_off);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        a.XS[c][t] = a.X[c][s];
        a.VP_new[c][t] = a.VP_cur[c][s];
    }
    a.R_new[t] = a.R_cur[s];
    a.T_new[t] = a.T_cur[s];
    a.ID_new[t] = a.ID_cur[s] - d.prev_cell_off + d.cell_off;
    a.slot_new[t] = k;
}

__global__ __launch_bounds__(BLOCK) void k_copy_u32(uint32_t n, const uint32_t* __restrict__ a,
                                                    uint32_t* __restrict__ b)
{
    const uint32_t s = blockIdx.x * BLOCK + threadIdx.x;
    if (s < n) b[s] = a[s];
}

// read-back of one slot: voxel order -> the slot's own id order, interleaved xyz.
template <typename VPT>
__global__ __launch_bounds__(BLOCK) void k_unpermute(uint32_t cell_off, uint32_t n,
                                                     const uint32_t* __restrict__ id,
                                                     const double* __restrict__ x0,
                                                     const double* __restrict__ x1,
                                                     const double* __restrict__ x2,
                                                     const VPT* __restrict__ v0,
                                                     const VPT* __restrict__ v1,
                                                     const VPT* __restrict__ v2,
                                                     double* __restrict__ pos,
                                                     double* __restrict__ vel)
{
    const uint32_t t = blockIdx.x * BLOCK + threadIdx.x;
    if (t >= n) return;
    const uint32_t s = cell_off + t;
    const size_t k = 3 * (size_t)(id[s] - cell_off);  // 64-bit: 3 * id passes 2^32 near 1.4e9 cells
    pos[k + 0] = x0[s];
    pos[k + 1] = x1[s];
    pos[k + 2] = x2[s];
    vel[k + 0] = (double)v0[s];
    vel[k + 1] = (double)v1[s];
    vel[k + 2] = (double)v2[s];
}

// The allocation-free entry point's input: positions and, when given, the history
// arrive as host-layout rows (x, y, z per cell) in the staging area; they go into the
// structure-of-arrays state of the first cell range of parity 0, with ids 0..n-1.
template <typename VPT>
__global__ __launch_bounds__(BLOCK) void k_load_cells(uint32_t n, const double* __restrict__ st, bool has_vprev,
                                                      double* __restrict__ x0, double* __restrict__ x1,
                                                      double* __restrict__ x2, uint32_t* __restrict__ id,
                                                      uint32_t* __restrict__ slot_of, VPT* __restrict__ v0,
                                                      VPT* __restrict__ v1, VPT* __restrict__ v2)
{
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const size_t k = 3 * (size_t)i;
    x0[i] = st[k + 0];
    x1[i] = st[k + 1];
    x2[i] = st[k + 2];
    id[i] = i;
    slot_of[i] = 0;
    const double* vp = st + 3 * (size_t)n;
    v0[i] = has_vprev ? (VPT)vp[k + 0] : (VPT)0;
    v1[i] = has_vprev ? (VPT)vp[k + 1] : (VPT)0;
    v2[i] = has_vprev ? (VPT)vp[k + 2] : (VPT)0;
}

// ------------------------------------------------------------------------ host side

inline uint32_t blocks_for(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

struct Layout {
    size_t X[3], XS[3], R[2], T[2], ID[2], VP[2][3], SH, XR, QS, slot_of, vid_cur, off, tmp_key, dtsum,
        tmp_src, vid_sorted, count, start, occ, hdr, tsum, stats, cadh, cadh_f, slots, stage, work, split;
    size_t total;
    bool xr = false;   // the FP64 records XR are kept
};

// One-type FP64 arenas keep a record (x, y, z, r) per cell, written by the gather, for the
// one-type kernels' evaluation: one 32-byte load per listed candidate instead of four
// gathers.  The 1M-cell tumour's step was 1.3-2.4% faster with it.  The two-type FP64
// kernels read the four arrays: with the record the 100k spheroid and the 256 small
// simulations run one at a time were about 2% slower (the gather writes 32 more bytes
// per cell, and these force kernels are latency-bound), and choosing between the two
// at run time cost the one-type kernel 4%.
bool fp64_records(const MechParams& p) { return p.precision == MECH_FP64 && p.n_types == 1; }

bool is_fp32(const MechParams& p) { return p.precision != MECH_FP64; }
// the float shadow's sign carries the cell type (the two-type FP32 kernels read no type)
bool sign_type(const MechParams& p) { return is_fp32(p) && p.n_types == 2; }

Layout make_layout(const MechParams& p, int64_t ncap, uint64_t vcap, int32_t scap)
{
    Layout L{};
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        size_t o = cur;
        cur += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t nn = (size_t)std::max<int64_t>(ncap, 1);
    const size_t vv = (size_t)std::max<uint64_t>(vcap, 1);
    const size_t vpb = is_fp32(p) ? sizeof(float) : sizeof(double);
    for (int c = 0; c < 3; ++c) L.X[c] = take(nn * 8);
    for (int c = 0; c < 3; ++c) L.XS[c] = take(nn * 8);
    for (int k = 0; k < 2; ++k) {
        L.R[k] = take(nn * 8);
        L.T[k] = take(nn * 4);
        L.ID[k] = take(nn * 4);
        for (int c = 0; c < 3; ++c) L.VP[k][c] = take(nn * vpb);
    }
    L.SH = take(is_fp32(p) ? nn * 16 : 0);   // read by the FP32 kernels only
    L.xr = fp64_records(p);
    L.XR = take(L.xr ? nn * 32 : 0);
    L.QS = take((nn + QS_PAD) * 8);        // a trip of the force kernel may read past the last cell
    L.slot_of = take(nn * 4);
    L.vid_cur = take(nn * 4);
    L.off = take(nn * 4);
    L.tmp_key = take(nn * 4);
    L.tmp_src = take(nn * 4);
    L.vid_sorted = take(nn * 4);
    L.count = take(XSUB * vv * 4);          // per bin
    L.start = take((XSUB * vv + 1) * 4);    // per bin, plus the total
    L.occ = take(vv * 4);                   // per voxel
    L.hdr = take(HDR_WORDS * 4);
    L.tsum = take((size_t)blocks_for(XSUB * vv, SCAN_TILE) * 8);
    L.stats = take(STAT_SLOTS * 16);
    L.cadh = take(64 * 8);
    L.cadh_f = take(64 * 4);
    L.slots = take((size_t)std::max(scap, 1) * sizeof(SlotDesc));
    L.stage = take(nn * 48);
    L.dtsum = take((size_t)blocks_for(nn, SCAN_TILE) * 8);
    L.work = take(BAL_ENTRIES * 4);
    L.split = take((N_XCD + 1) * 4);
    L.total = cur;
    return L;
}

// Parameters shared by the slots of a batch (the domain fields are not used here).
int validate_physics(const MechParams* p)
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
    return MECH_OK;
}

// Units per um of the quantised shadow: the largest power of two S with h S <= 2^13.
double quant_scale(double h) { return std::ldexp(1.0, (int)std::floor(std::log2(8192.0 / h))); }

int validate_domain(const double lo[3], const double hi[3], double h, int32_t dims[3], uint64_t* V)
{
    // The quantised shadow rounds x S to an integer: it must stay exact in a double (and
    // S finite in a float).  The prefilter takes its threshold t = (reach_i + reach_j
    // + Q_MARGIN + q_pad) units as an int16 and squares it in 32 bits, so t must stay
    // below 2^15: each reach is at most alpha r_max S <= h S / 2 <= 2^12 units (the voxel
    // holds 2 alpha r_max), and q_pad = ceil(2^-20 P S) grows with the largest coordinate P.
    {
        const double S = quant_scale(h);
        double pm = 0.0;
        for (int a = 0; a < 3; ++a) pm = std::max(pm, std::max(std::fabs(lo[a]), std::fabs(hi[a])));
        if (!(S < 0x1p100)) return fail(MECH_E_INVALID, "voxel_size %.17g is too small", h);
        if (!(pm * S < 0x1p52) || !(std::ceil(pm * S * 0x1p-20) + 2.0 * 4096.0 + (double)Q_MARGIN < 32768.0))
            return fail(MECH_E_INVALID, "domain coordinates up to %.17g um are too large for voxel_size %.17g "
                        "(the prefilter's margin would overflow)", pm, h);
    }
    uint64_t v = 1;
    for (int a = 0; a < 3; ++a) {
        if (!(std::isfinite(lo[a]) && std::isfinite(hi[a]) && hi[a] >= lo[a]))
            return fail(MECH_E_INVALID, "domain axis %d: need finite lo <= hi", a);
        double cells = std::ceil((hi[a] - lo[a]) / h);
        if (cells > 2147483647.0) return fail(MECH_E_INVALID, "too many voxels on axis %d", a);
        dims[a] = std::max(1, (int)cells);
        v *= (uint64_t)dims[a];
    }
    if (v >= (uint64_t(1) << 30)) return fail(MECH_E_INVALID, "grid of %llu voxels is too large", (unsigned long long)v);
    *V = v;
    return MECH_OK;
}

int validate_cells(const MechParams* p, const double lo[3], const double hi[3], int64_t n,
                   const double* pos, const double* radius, const int32_t* type,
                   const double* vprev, double* rmax_out)
{
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(MECH_E_INVALID, "n_cells %lld out of range", (long long)n);
    if (n > 0 && (!pos || !radius)) return fail(MECH_E_INVALID, "pos and radius are required");
    double rmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double r = radius[i];
        if (!(std::isfinite(r) && r > 0)) return fail(MECH_E_INVALID, "radius[%lld] must be finite and > 0", (long long)i);
        rmax = std::max(rmax, r);
        for (int a = 0; a < 3; ++a) {
            double x = pos[3 * i + a];
            if (!std::isfinite(x)) return fail(MECH_E_INVALID, "pos[%lld] is not finite", (long long)i);
            if (x < lo[a] || x > hi[a])
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
    *rmax_out = rmax;
    return MECH_OK;
}

// Host view of one slot.
struct HostSlot {
    SlotDesc d{};
    bool used = false;       // holds a simulation (running, frozen or retired)
    bool retired = false;    // cells still in the arena until the next repack
    bool reported = false;   // completion already returned by batch_poll
    int64_t steps_total = 0; // steps requested (< 0: no limit)
    hipEvent_t done = nullptr;  // recorded after the step that froze the slot
    bool done_recorded = false;
};

}  // namespace

struct MechBatch {
    MechParams prm{};
    PhysArgs phys{};
    int device = 0;
    hipStream_t stream = nullptr, copy_stream = nullptr;
    bool own_stream = false;
    hipEvent_t copy_done = nullptr;
    hipEvent_t clock = nullptr;           // batch_mark_clock's reference point
    bool clock_marked = false;
    char* arena = nullptr;
    bool own_arena = false;
    Layout L{};
    int64_t cap_cells = 0, cap_voxels = 0;
    int32_t cap_slots = 0;
    uint32_t n_cells = 0, n_voxels = 0;   // host mirror of the header
    std::vector<HostSlot> slots;
    std::vector<int32_t> order;           // used slots in arena order
    int parity = 0;
    int64_t steps = 0;
    int32_t cus = 256;                    // compute units of the device
    MechTuning tune{0, 1, 8, 0, 0};       // force-kernel launch configuration
    // locality study: reorder (gather) every reorder_every steps, 0 = never
    int32_t reorder_every = 1;
    // growing populations: division probability per cell and step, draw seed
    double p_div = 0.0;
    uint64_t div_seed = 0;
    double p_death = 0.0;                 // dying populations: death probability per step
    bool step_start = false;              // the binning being enqueued starts a step
    bool growing = false;                 // the device may hold more cells than the host mirror
    int64_t reorder_phase = 0;            // steps since the mode was set
    bool last_gather = true;              // the last binning reordered the cells
    bool graphs_ready = false;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipGraphExec_t gexec_inplace[2] = {nullptr, nullptr};
    hipGraphExec_t gexec_run[2] = {nullptr, nullptr};  // RUN_STEPS reordering steps

    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(arena + off); }
};

struct MechPopulation {
    MechBatch* b = nullptr;
    int64_t n = 0;
};

namespace {

// ------------------------------------------------------------------------ enqueue

// Launch grids are fixed per batch (the captured graph never changes) and bounded: the
// kernels loop over what the device header says is live, so a large arena costs no
// empty workgroups.
constexpr uint32_t CELL_GRID_MAX = 8192;   // workgroups of 256 for per-cell kernels
constexpr uint32_t TILE_GRID_MAX = 2048;   // workgroups for the voxel-scan kernels

uint32_t cell_grid(const MechBatch* B)
{
    return std::max<uint32_t>(1, std::min<uint32_t>(blocks_for((uint64_t)B->cap_cells, BLOCK), CELL_GRID_MAX));
}

bool force_balanced(const MechBatch* B);

// a1..a3 and the scatter of a4 (sorted slots of the cells, before the rank by id); with
// `balance`, k_bin also cuts the next force launch's XCD runs from the last one's work
void enqueue_keys(MechBatch* B, bool balance)
{
    const Layout& L = B->L;
    const int cur = B->parity;
    const uint32_t nbc = cell_grid(B);
    const uint32_t nbt = std::min<uint32_t>(blocks_for((uint64_t)B->cap_voxels * XSUB, SCAN_TILE), TILE_GRID_MAX);
    const uint32_t* hdr = B->at<uint32_t>(L.hdr);
    hipLaunchKernelGGL(k_bin, dim3(nbc + (balance ? 1 : 0)), dim3(BLOCK), 0, B->stream, B->at<double>(L.X[0]),
                       B->at<double>(L.X[1]), B->at<double>(L.X[2]), B->at<uint32_t>(L.slot_of),
                       B->at<SlotDesc>(L.slots), B->at<uint32_t>(L.hdr), B->at<uint32_t>(L.count),
                       B->at<uint32_t>(L.vid_cur), B->at<uint32_t>(L.off), (uint32_t)B->cap_slots,
                       B->step_start ? 1 : 0, balance ? B->at<uint32_t>(L.work) : nullptr,
                       B->at<uint32_t>(L.split));
    hipLaunchKernelGGL(k_scan_reduce, dim3(nbt), dim3(BLOCK), 0, B->stream, B->at<uint32_t>(L.count), hdr,
                       B->at<uint64_t>(L.tsum));
    if (blocks_for((uint64_t)B->cap_voxels * XSUB, SCAN_TILE) <= FUSED_SCAN_TILES) {
        hipLaunchKernelGGL(k_scan_down<true>, dim3(nbt), dim3(BLOCK), 0, B->stream, B->at<uint32_t>(L.count),
                           B->at<uint32_t>(L.hdr), B->at<uint64_t>(L.tsum), B->at<uint32_t>(L.start),
                           B->at<uint32_t>(L.occ));
    } else {
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(TOP_BLOCK), 0, B->stream, B->at<uint64_t>(L.tsum),
                           B->at<uint32_t>(L.start), B->at<uint32_t>(L.hdr));
        hipLaunchKernelGGL(k_scan_down<false>, dim3(nbt), dim3(BLOCK), 0, B->stream, B->at<uint32_t>(L.count),
                           B->at<uint32_t>(L.hdr), B->at<uint64_t>(L.tsum), B->at<uint32_t>(L.start),
                           B->at<uint32_t>(L.occ));
    }
    hipLaunchKernelGGL(k_scatter, dim3(nbc), dim3(BLOCK), 0, B->stream, hdr, B->at<uint32_t>(L.vid_cur),
                       B->at<uint32_t>(L.off), B->at<uint32_t>(L.start), B->at<uint32_t>(L.ID[cur]),
                       B->at<uint32_t>(L.tmp_key), B->at<uint32_t>(L.tmp_src));
}

// A single small population takes the one-launch path (k_bin_small).
bool small_binning(const MechBatch* B)
{
    return B->cap_slots == 1 && B->cap_cells <= (int64_t)SMALL_CELLS &&
           (int64_t)XSUB * B->cap_voxels <= (int64_t)SMALL_BINS;
}

template <typename VPT>
void enqueue_binning(MechBatch* B)
{
    const Layout& L = B->L;
    const int cur = B->parity, nxt = cur ^ 1;
    const uint32_t nbc = cell_grid(B);
    const uint32_t* hdr = B->at<uint32_t>(L.hdr);
    if (!small_binning(B)) enqueue_keys(B, force_balanced(B));
    GatherArgs<VPT> g{};
    for (int c = 0; c < 3; ++c) {
        g.X[c] = B->at<double>(L.X[c]);
        g.XS[c] = B->at<double>(L.XS[c]);
        g.VP_cur[c] = B->at<VPT>(L.VP[cur][c]);
        g.VP_new[c] = B->at<VPT>(L.VP[nxt][c]);
    }
    g.R_cur = B->at<double>(L.R[cur]);
    g.R_new = B->at<double>(L.R[nxt]);
    g.T_cur = B->at<int32_t>(L.T[cur]);
    g.T_new = B->at<int32_t>(L.T[nxt]);
    g.ID_new = B->at<uint32_t>(L.ID[nxt]);
    g.SH = is_fp32(B->prm) ? B->at<float4>(L.SH) : nullptr;
    g.XR = L.xr ? B->at<double4>(L.XR) : nullptr;
    g.QS = B->at<uint2>(L.QS);
    g.sign_type = sign_type(B->prm) ? 1 : 0;
    g.slot_of = B->at<uint32_t>(L.slot_of);
    g.slots = B->at<SlotDesc>(L.slots);
    g.alpha = B->phys.alpha;
    g.vid_cur = B->at<uint32_t>(L.vid_cur);
    g.tmp_key = B->at<uint32_t>(L.tmp_key);
    g.tmp_src = B->at<uint32_t>(L.tmp_src);
    g.voxel_start = B->at<uint32_t>(L.start);
    g.vid_sorted = B->at<uint32_t>(L.vid_sorted);
    if (small_binning(B))
        hipLaunchKernelGGL(k_bin_small<VPT>, dim3(1), dim3(SMALL_BLOCK), 0, B->stream, B->at<uint32_t>(L.slot_of),
                           B->at<SlotDesc>(L.slots), B->at<uint32_t>(L.hdr), B->at<uint32_t>(L.ID[cur]),
                           B->at<uint32_t>(L.vid_cur), B->at<uint32_t>(L.start), B->at<uint32_t>(L.occ), g,
                           (uint32_t)B->cap_slots, B->step_start ? 1 : 0);
    else
        hipLaunchKernelGGL(k_rank_gather<VPT>, dim3(nbc), dim3(BLOCK), 0, B->stream, hdr, g);
}

// Workgroups of a per-cell force kernel: one per WPB*64 cells of the arena's capacity,
// at most 32768 wave64s in total, or tune.blocks_per_cu per compute unit.  The kernels
// loop over the live cells, so any count is correct; it only sets how work is dealt.
uint32_t force_cell_grid(const MechBatch* B, int wpb)
{
    const uint32_t tiles = std::max<uint32_t>(1, blocks_for((uint64_t)B->cap_cells, (uint32_t)wpb * WAVE));
    const uint32_t cap = B->tune.blocks_per_cu ? (uint32_t)B->cus * (uint32_t)B->tune.blocks_per_cu
                                               : 32768u / (uint32_t)wpb;
    return std::min(tiles, cap);
}

// Whether the step's force launch records its waves' durations and takes work-balanced
// XCD runs: the per-cell list kernel, with a grid that fills every resident slot at
// least once (with fewer workgroups, a longer run would make some of them take two
// tiles in turn).
bool force_balanced(const MechBatch* B)
{
    if (B->prm.flags & (MECH_FLAG_SIMPLE_FORCE | MECH_FLAG_VOXEL_FORCE)) return false;
    const int w = B->tune.block_waves;
    const uint32_t wpb = (w == 1 || w == 2 || w == 8) ? (uint32_t)w : 4u;
    return force_cell_grid(B, (int)wpb) >= (uint32_t)B->cus * (32u / wpb);
}

template <int PREC, bool MULTI, typename VPT, int WPB, int LIST, bool PRUNE>
void launch_cells_p(MechBatch* B, const ForceArgs<VPT>& args)
{
    const dim3 grid(force_cell_grid(B, WPB)), block(WPB * WAVE);
    // a ring entry of a single-type trip of 8 holds candidate indices below 2^24: larger
    // arenas take trips of 4 (same results: the candidates are listed and evaluated in the
    // same order)
    const int unroll = !MULTI && LIST < 32 && B->tune.unroll == 8 && B->cap_cells >= ((int64_t)1 << 24)
                           ? 4 : B->tune.unroll;
    ForceArgs<VPT> a = args;
    if (!force_balanced(B)) {
        a.work = nullptr;
        a.split = nullptr;
    }
    switch (unroll) {
    case 2:
        hipLaunchKernelGGL((k_force_cells<PREC, MULTI, VPT, WPB, 2, LIST, false, PRUNE>), grid, block, 0, B->stream,
                           B->phys, a);
        break;
    case 8:
        hipLaunchKernelGGL((k_force_cells<PREC, MULTI, VPT, WPB, 8, LIST, false, PRUNE>), grid, block, 0, B->stream,
                           B->phys, a);
        break;
    default:
        hipLaunchKernelGGL((k_force_cells<PREC, MULTI, VPT, WPB, 4, LIST, false, PRUNE>), grid, block, 0, B->stream,
                           B->phys, a);
        break;
    }
}

template <int PREC, bool MULTI, typename VPT, int WPB, int LIST>
void launch_cells_l(MechBatch* B, const ForceArgs<VPT>& a)
{
    if (B->prm.flags & MECH_FLAG_PRUNED_FORCE)
        launch_cells_p<PREC, MULTI, VPT, WPB, LIST, true>(B, a);
    else
        launch_cells_p<PREC, MULTI, VPT, WPB, LIST, false>(B, a);
}

template <int PREC, bool MULTI, typename VPT, int WPB>
void launch_cells_w(MechBatch* B, const ForceArgs<VPT>& a)
{
    // the ring's packed entries hold candidate indices below 2^28: larger arenas take
    // the 32-entry list
    const int len = (B->tune.list_len == 16 || B->tune.list_len == 0) && B->cap_cells >= ((int64_t)1 << 28)
                        ? 32 : B->tune.list_len;
    switch (len) {
    case 32: launch_cells_l<PREC, MULTI, VPT, WPB, 32>(B, a); break;
    case 64:
        // 8 waves with 64-entry lists would take more LDS than a CU has (set_tuning
        // rejects the pair)
        if constexpr (WPB <= 4) launch_cells_l<PREC, MULTI, VPT, WPB, 64>(B, a);
        break;
    default: launch_cells_l<PREC, MULTI, VPT, WPB, 16>(B, a); break;
    }
}

template <int PREC, bool MULTI, typename VPT>
void launch_cells(MechBatch* B, const ForceArgs<VPT>& a)
{
    switch (B->tune.block_waves) {
    case 1: launch_cells_w<PREC, MULTI, VPT, 1>(B, a); break;
    case 2: launch_cells_w<PREC, MULTI, VPT, 2>(B, a); break;
    case 8: launch_cells_w<PREC, MULTI, VPT, 8>(B, a); break;
    default: launch_cells_w<PREC, MULTI, VPT, 4>(B, a); break;
    }
}

template <int PREC, bool MULTI, typename VPT, int WPB>
void launch_rows_w(MechBatch* B, const ForceArgs<VPT>& a)
{
    hipLaunchKernelGGL((k_force_rows<PREC, MULTI, VPT, WPB>), dim3(force_cell_grid(B, WPB)), dim3(WPB * WAVE), 0,
                       B->stream, B->phys, a);
}

template <int PREC, bool MULTI, typename VPT>
void launch_rows(MechBatch* B, const ForceArgs<VPT>& a)
{
    switch (B->tune.block_waves) {
    case 1: launch_rows_w<PREC, MULTI, VPT, 1>(B, a); break;
    case 2: launch_rows_w<PREC, MULTI, VPT, 2>(B, a); break;
    case 8: launch_rows_w<PREC, MULTI, VPT, 8>(B, a); break;
    default: launch_rows_w<PREC, MULTI, VPT, 4>(B, a); break;
    }
}

template <int PREC, typename VPT>
void enqueue_force(MechBatch* B, int parity_after_sort)
{
    const Layout& L = B->L;
    const int p = parity_after_sort;
    ForceArgs<VPT> a{};
    for (int c = 0; c < 3; ++c) {
        a.XS[c] = B->at<double>(L.XS[c]);
        a.X[c] = B->at<double>(L.X[c]);
        a.VP[c] = B->at<VPT>(L.VP[p][c]);
    }
    a.R = B->at<double>(L.R[p]);
    a.T = B->at<int32_t>(L.T[p]);
    a.SH = is_fp32(B->prm) ? B->at<float4>(L.SH) : nullptr;
    a.XR = L.xr ? B->at<double4>(L.XR) : nullptr;
    a.QS = B->at<uint2>(L.QS);
    a.vid_sorted = B->at<uint32_t>(L.vid_sorted);
    a.voxel_start = B->at<uint32_t>(L.start);
    a.slot_of = B->at<uint32_t>(L.slot_of);
    a.slots = B->at<SlotDesc>(L.slots);
    a.hdr = B->at<uint32_t>(L.hdr);
    a.cadh = B->at<double>(L.cadh);
    a.cadh_f = B->at<float>(L.cadh_f);
    a.stats = B->at<unsigned long long>(L.stats);
    const bool multi = B->prm.n_types > 1;
    if (B->prm.flags & MECH_FLAG_SIMPLE_FORCE) {
        if (multi)
            launch_rows<PREC, true, VPT>(B, a);
        else
            launch_rows<PREC, false, VPT>(B, a);
    } else if (B->prm.flags & MECH_FLAG_VOXEL_FORCE) {
        const uint32_t* occ = B->at<uint32_t>(L.occ);
        const uint32_t grid = (uint32_t)B->cus * (uint32_t)(B->tune.blocks_per_cu ? B->tune.blocks_per_cu : 4);
        if (multi)
            hipLaunchKernelGGL((k_force_lds<PREC, true, VPT>), dim3(grid), dim3(FL_WAVES * WAVE), 0,
                               B->stream, B->phys, a, occ);
        else
            hipLaunchKernelGGL((k_force_lds<PREC, false, VPT>), dim3(grid), dim3(FL_WAVES * WAVE), 0,
                               B->stream, B->phys, a, occ);
    } else {
        a.work = B->at<uint32_t>(L.work);
        a.split = B->at<uint32_t>(L.split);
        if (multi)
            launch_cells<PREC, true, VPT>(B, a);
        else
            launch_cells<PREC, false, VPT>(B, a);
    }
}

void enqueue_binning_any(MechBatch* B)
{
    if (is_fp32(B->prm))
        enqueue_binning<float>(B);
    else
        enqueue_binning<double>(B);
}

void enqueue_force_any(MechBatch* B, int parity_after_sort)
{
    switch (B->prm.precision) {
    case MECH_FP64: enqueue_force<0, double>(B, parity_after_sort); break;
    case MECH_FP32: enqueue_force<1, float>(B, parity_after_sort); break;
    default: enqueue_force<2, float>(B, parity_after_sort); break;
    }
}

// ------------------------------------------------------------------------ cells left in place

// The locality study: binning as usual, but the cells stay in their storage order; the
// force kernel takes the cells in that order and reads the candidates of the sorted
// order through perm (which aliases `off`, free once a4's scatter has used it).
template <int PREC, typename VPT>
void enqueue_force_inplace(MechBatch* B)
{
    const Layout& L = B->L;
    const int cur = B->parity;
    ForceArgs<VPT> a{};
    for (int c = 0; c < 3; ++c) {
        a.XS[c] = B->at<double>(L.X[c]);   // positions, storage order
        a.X[c] = B->at<double>(L.XS[c]);   // new positions, storage order
        a.VP[c] = B->at<VPT>(L.VP[cur][c]);
    }
    a.R = B->at<double>(L.R[cur]);
    a.T = B->at<int32_t>(L.T[cur]);
    a.SH = is_fp32(B->prm) ? B->at<float4>(L.SH) : nullptr;
    a.XR = L.xr ? B->at<double4>(L.XR) : nullptr;
    a.QS = B->at<uint2>(L.QS);
    a.vid_sorted = B->at<uint32_t>(L.vid_cur);
    a.voxel_start = B->at<uint32_t>(L.start);
    a.slot_of = B->at<uint32_t>(L.slot_of);
    a.slots = B->at<SlotDesc>(L.slots);
    a.hdr = B->at<uint32_t>(L.hdr);
    a.cadh = B->at<double>(L.cadh);
    a.cadh_f = B->at<float>(L.cadh_f);
    a.stats = B->at<unsigned long long>(L.stats);
    a.perm = B->at<uint32_t>(L.off);
    const dim3 grid(force_cell_grid(B, 4)), block(4 * WAVE);
    if (B->prm.n_types > 1)
        hipLaunchKernelGGL((k_force_cells<PREC, true, VPT, 4, 4, 16, true>), grid, block, 0, B->stream, B->phys, a);
    else
        hipLaunchKernelGGL((k_force_cells<PREC, false, VPT, 4, 4, 16, true>), grid, block, 0, B->stream, B->phys, a);
}

// a1..a4 without the reorder: keys, scan, scatter, perm (and the float shadow first).
void enqueue_binning_inplace(MechBatch* B)
{
    const Layout& L = B->L;
    const int cur = B->parity;
    const uint32_t nbc = cell_grid(B);
    const uint32_t* hdr = B->at<uint32_t>(L.hdr);
    hipLaunchKernelGGL(k_shadow, dim3(nbc), dim3(BLOCK), 0, B->stream, hdr, B->at<double>(L.X[0]),
                       B->at<double>(L.X[1]), B->at<double>(L.X[2]), B->at<double>(L.R[cur]),
                       is_fp32(B->prm) ? B->at<float4>(L.SH) : nullptr, B->at<uint2>(L.QS),
                       B->at<uint32_t>(L.slot_of),
                       B->at<SlotDesc>(L.slots), B->phys.alpha, B->at<int32_t>(L.T[cur]),
                       sign_type(B->prm) ? 1 : 0, L.xr ? B->at<double4>(L.XR) : nullptr);
    enqueue_keys(B, false);
    hipLaunchKernelGGL(k_rank_perm, dim3(nbc), dim3(BLOCK), 0, B->stream, hdr, B->at<uint32_t>(L.vid_cur),
                       B->at<uint32_t>(L.tmp_key), B->at<uint32_t>(L.tmp_src), B->at<uint32_t>(L.start),
                       B->at<uint32_t>(L.off));
}

void enqueue_force_inplace_any(MechBatch* B)
{
    const Layout& L = B->L;
    switch (B->prm.precision) {
    case MECH_FP64: enqueue_force_inplace<0, double>(B); break;
    case MECH_FP32: enqueue_force_inplace<1, float>(B); break;
    default: enqueue_force_inplace<2, float>(B); break;
    }
    hipLaunchKernelGGL(k_commit, dim3(cell_grid(B)), dim3(BLOCK), 0, B->stream, B->at<uint32_t>(L.hdr),
                       B->at<double>(L.XS[0]), B->at<double>(L.XS[1]), B->at<double>(L.XS[2]),
                       B->at<double>(L.X[0]), B->at<double>(L.X[1]), B->at<double>(L.X[2]));
}

void enqueue_step_end(MechBatch* B)
{
    hipLaunchKernelGGL(k_step_end, dim3(blocks_for((uint64_t)B->cap_slots, BLOCK)), dim3(BLOCK), 0, B->stream,
                       B->at<SlotDesc>(B->L.slots), (uint32_t)B->cap_slots, B->at<uint32_t>(B->L.hdr));
}

// Division after the walls (growing populations): `buf` is the buffer pair that holds
// the step's cells (the gathered one after a reorder, the current one in place).
void enqueue_division(MechBatch* B, int buf)
{
    if (!(B->p_div > 0.0)) return;
    const Layout& L = B->L;
    DivArgs a{};
    for (int c = 0; c < 3; ++c) {
        a.X[c] = B->at<double>(L.X[c]);
        a.VP[c] = B->arena + L.VP[buf][c];
    }
    a.R = B->at<double>(L.R[buf]);
    a.T = B->at<int32_t>(L.T[buf]);
    a.ID = B->at<uint32_t>(L.ID[buf]);
    a.slot_of = B->at<uint32_t>(L.slot_of);
    a.slots = B->at<SlotDesc>(L.slots);
    a.hdr = B->at<uint32_t>(L.hdr);
    a.flag = B->at<uint32_t>(L.tmp_key);   // free once a4 has used it
    a.tsum = B->at<uint64_t>(L.dtsum);
    a.seed = B->div_seed;
    a.p_div = B->p_div;
    a.capacity = (uint32_t)B->cap_cells;
    a.vp_bytes = is_fp32(B->prm) ? 4u : 8u;
    const uint32_t nbc = cell_grid(B);
    const uint32_t nbt = std::min<uint32_t>(blocks_for((uint64_t)B->cap_cells, SCAN_TILE), TILE_GRID_MAX);
    hipLaunchKernelGGL(k_div_mark, dim3(nbc), dim3(BLOCK), 0, B->stream, a);
    hipLaunchKernelGGL(k_div_scan_reduce, dim3(nbt), dim3(BLOCK), 0, B->stream, a);
    hipLaunchKernelGGL(k_div_scan_top, dim3(1), dim3(BLOCK), 0, B->stream, a);
    hipLaunchKernelGGL(k_div_scan_down, dim3(nbt), dim3(BLOCK), 0, B->stream, a);
    hipLaunchKernelGGL(k_div_apply, dim3(nbc), dim3(BLOCK), 0, B->stream, a);
    hipLaunchKernelGGL(k_div_commit, dim3(1), dim3(1), 0, B->stream, a);
}

// Death after division (dying populations): `buf` as for division; the survivors are
// gathered into the other buffer pair and the positions' gathered copy XS (both free
// once the force kernel has run), then copied back.
void enqueue_death(MechBatch* B, int buf)
{
    if (!(B->p_death > 0.0)) return;
    const Layout& L = B->L;
    DivArgs a{};
    for (int c = 0; c < 3; ++c) {
        a.X[c] = B->at<double>(L.X[c]);
        a.VP[c] = B->arena + L.VP[buf][c];
        a.X_alt[c] = B->at<double>(L.XS[c]);
        a.VP_alt[c] = B->arena + L.VP[buf ^ 1][c];
    }
    a.R = B->at<double>(L.R[buf]);
    a.T = B->at<int32_t>(L.T[buf]);
    a.ID = B->at<uint32_t>(L.ID[buf]);
    a.R_alt = B->at<double>(L.R[buf ^ 1]);
    a.T_alt = B->at<int32_t>(L.T[buf ^ 1]);
    a.ID_alt = B->at<uint32_t>(L.ID[buf ^ 1]);
    a.slot_of = B->at<uint32_t>(L.slot_of);
    a.slots = B->at<SlotDesc>(L.slots);
    a.hdr = B->at<uint32_t>(L.hdr);
    a.flag = B->at<uint32_t>(L.tmp_key);
    a.tsum = B->at<uint64_t>(L.dtsum);
    a.seed = B->div_seed;
    a.p_death = B->p_death;
    a.vp_bytes = is_fp32(B->prm) ? 4u : 8u;
    const uint32_t nbc = cell_grid(B);
    const uint32_t nbt = std::min<uint32_t>(blocks_for((uint64_t)B->cap_cells, SCAN_TILE), TILE_GRID_MAX);
    hipLaunchKernelGGL(k_die_mark, dim3(nbc), dim3(BLOCK), 0, B->stream, a);
    hipLaunchKernelGGL(k_div_scan_reduce, dim3(nbt), dim3(BLOCK), 0, B->stream, a);
    hipLaunchKernelGGL(k_div_scan_top, dim3(1), dim3(BLOCK), 0, B->stream, a);
    hipLaunchKernelGGL(k_div_scan_down, dim3(nbt), dim3(BLOCK), 0, B->stream, a);
    hipLaunchKernelGGL(k_die_move, dim3(nbc), dim3(BLOCK), 0, B->stream, a);
    hipLaunchKernelGGL(k_die_back, dim3(nbc), dim3(BLOCK), 0, B->stream, a);
    hipLaunchKernelGGL(k_die_commit, dim3(1), dim3(1), 0, B->stream, a);
}

// One full step a1..a7 from `parity`; flips nothing on the host.  gather: reorder the
// cells (the default); otherwise leave them in place (the step keeps the parity).
void enqueue_step(MechBatch* B, int parity, bool gather = true)
{
    const int saved = B->parity;
    B->parity = parity;
    B->step_start = true;   // the first binning kernel does the step's bookkeeping
    if (gather) {
        enqueue_binning_any(B);
        B->step_start = false;
        enqueue_force_any(B, parity ^ 1);
    } else {
        enqueue_binning_inplace(B);
        B->step_start = false;
        enqueue_force_inplace_any(B);
    }
    enqueue_division(B, gather ? parity ^ 1 : parity);
    enqueue_death(B, gather ? parity ^ 1 : parity);
    B->parity = saved;
}

bool gather_now(const MechBatch* B)
{
    if (B->reorder_every == 1) return true;
    if (B->reorder_every == 0) return false;
    return B->reorder_phase % B->reorder_every == 0;
}

int sync_check(MechBatch* B)
{
    HIP_TRY(hipStreamSynchronize(B->stream));
    HIP_TRY(hipGetLastError());
    return MECH_OK;
}

int drop_graphs(MechBatch* B)
{
    for (int p = 0; p < 2; ++p) {
        if (B->gexec[p]) {
            (void)hipGraphExecDestroy(B->gexec[p]);
            B->gexec[p] = nullptr;
        }
        if (B->gexec_inplace[p]) {
            (void)hipGraphExecDestroy(B->gexec_inplace[p]);
            B->gexec_inplace[p] = nullptr;
        }
        if (B->gexec_run[p]) {
            (void)hipGraphExecDestroy(B->gexec_run[p]);
            B->gexec_run[p] = nullptr;
        }
    }
    B->graphs_ready = false;
    return MECH_OK;
}

// One graph per parity for reordering steps and, when cells may be left in place, one
// per parity for those steps.  When every step reorders, also one per parity for a run
// of RUN_STEPS steps: small populations are bound by the host's launch rate, and one
// launch per run instead of per step takes most of it away.
constexpr int RUN_STEPS = 8;
static_assert(RUN_STEPS % 2 == 0, "a run ends on the parity it started from");

int build_graphs(MechBatch* B)
{
    for (int kind = 0; kind < 3; ++kind) {
        if (kind == 1 && B->reorder_every == 1) continue;
        if (kind == 2 && B->reorder_every != 1) break;
        for (int p = 0; p < 2; ++p) {
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
            if (kind == 2)
                for (int i = 0; i < RUN_STEPS; ++i) enqueue_step(B, p ^ (i & 1), true);
            else
                enqueue_step(B, p, kind == 0);
            hipError_t e = hipStreamEndCapture(B->stream, &g);
            if (e != hipSuccess) return fail(MECH_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
            hipGraphExec_t* dst = kind == 0 ? &B->gexec[p] : kind == 1 ? &B->gexec_inplace[p] : &B->gexec_run[p];
            e = hipGraphInstantiate(dst, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return fail(MECH_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
        }
    }
    B->graphs_ready = true;
    return MECH_OK;
}

void release(MechBatch* B)
{
    if (!B) return;
    (void)hipSetDevice(B->device);
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    if (B->copy_stream) (void)hipStreamSynchronize(B->copy_stream);
    drop_graphs(B);
    for (auto& s : B->slots)
        if (s.done) (void)hipEventDestroy(s.done);
    if (B->copy_done) (void)hipEventDestroy(B->copy_done);
    if (B->clock) (void)hipEventDestroy(B->clock);
    if (B->own_arena && B->arena) (void)hipFree(B->arena);
    if (B->copy_stream) (void)hipStreamDestroy(B->copy_stream);
    if (B->own_stream && B->stream) (void)hipStreamDestroy(B->stream);
    delete B;
}

void push_header(MechBatch* B)
{
    hipLaunchKernelGGL(k_set_header, dim3(1), dim3(1), 0, B->stream, B->at<uint32_t>(B->L.hdr), B->n_cells,
                       B->n_voxels);
}

void push_slot(MechBatch* B, int32_t id)
{
    hipLaunchKernelGGL(k_set_slot, dim3(1), dim3(1), 0, B->stream, B->at<SlotDesc>(B->L.slots), (uint32_t)id,
                       B->slots[id].d);
}

// The physics constants the kernels take, in both precisions.
PhysArgs phys_args(const MechParams& p)
{
    PhysArgs a{};
    a.dt = p.dt;
    a.c_rep = p.c_rep;
    a.alpha = p.rel_adh_distance;
    a.c_adh0 = p.c_adh[0];
    a.c_rep_f = (float)p.c_rep;
    a.alpha_f = (float)p.rel_adh_distance;
    a.inv_alpha_f = 1.0f / a.alpha_f;
    a.c_adh0_f = (float)p.c_adh[0];
    a.n_types = p.n_types;
    return a;
}

// The descriptor of a simulation of n cells (largest radius rmax) on a grid of dims
// voxels over [lo, hi], placed at the given cell and voxel offsets of the arena.
SlotDesc slot_desc(const MechParams& prm, const double lo[3], const double hi[3], const int32_t dims[3],
                   double rmax, int64_t n, int64_t n_steps, bool has_vprev, uint32_t cell_off, uint32_t voxel_off)
{
    SlotDesc d{};
    for (int a = 0; a < 3; ++a) {
        d.lo[a] = lo[a];
        d.hi[a] = hi[a];
    }
    d.inv_h = 1.0 / prm.voxel_size;
    d.r_max = rmax;
    d.r_max_f = (float)rmax;
    // the largest power of two with h S <= 2^13, and the margin for float positions
    // (2^-20 P S units, P the largest coordinate magnitude of the domain)
    d.q_scale = (float)quant_scale(prm.voxel_size);
    {
        double pm = 0.0;
        for (int a = 0; a < 3; ++a) pm = std::max(pm, std::max(std::fabs(lo[a]), std::fabs(hi[a])));
        d.q_pad = (float)std::ceil(pm * (double)d.q_scale * 0x1p-20);
    }
    d.nx = dims[0];
    d.ny = dims[1];
    d.nz = dims[2];
    d.voxel_off = voxel_off;
    d.cell_off = cell_off;
    d.prev_cell_off = d.cell_off;
    d.n_cells = (uint32_t)n;
    d.steps_left = n_steps < 0 ? -1 : (int32_t)std::min<int64_t>(n_steps, INT32_MAX);
    d.euler = (prm.ab2_start == MECH_AB2_EULER_START && !has_vprev) ? 1 : 0;
    return d;
}

int create_batch_impl(const MechParams* params, int64_t max_cells, int64_t max_voxels, int32_t max_slots,
                      void* stream, void* workspace, int64_t ws_bytes, MechBatch** out)
{
    if (!out) return fail(MECH_E_INVALID, "out is NULL");
    *out = nullptr;
    int rc = validate_physics(params);
    if (rc) return rc;
    if (max_cells < 0 || max_cells >= (int64_t(1) << 31)) return fail(MECH_E_INVALID, "max_cells out of range");
    if (max_voxels < 1 || max_voxels >= (int64_t(1) << 30)) return fail(MECH_E_INVALID, "max_voxels out of range");
    if (max_slots < 1 || max_slots > 65536) return fail(MECH_E_INVALID, "max_slots out of range");

    MechBatch* B = new MechBatch();
    B->prm = *params;
    B->cap_cells = max_cells;
    B->cap_voxels = max_voxels;
    B->cap_slots = max_slots;
    B->slots.resize((size_t)max_slots);
    B->phys = phys_args(*params);
    B->L = make_layout(*params, max_cells, (uint64_t)max_voxels, max_slots);
    auto bail = [&](int code) {
        release(B);
        return code;
    };
    if (hipGetDevice(&B->device) != hipSuccess) return bail(fail(MECH_E_DEVICE, "no HIP device"));
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, B->device) != hipSuccess || cus < 1)
            cus = 256;
        B->cus = cus;
    }
    if (stream) {
        B->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(MECH_E_DEVICE, "hipStreamCreate failed"));
        B->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&B->copy_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&B->copy_done, hipEventDisableTiming) != hipSuccess)
        return bail(fail(MECH_E_DEVICE, "stream or event creation failed"));
    // completion events keep timing: batch_slot_done_ms measures them against the clock mark
    for (auto& s : B->slots)
        if (hipEventCreate(&s.done) != hipSuccess) return bail(fail(MECH_E_DEVICE, "hipEventCreate failed"));
    if (hipEventCreate(&B->clock) != hipSuccess) return bail(fail(MECH_E_DEVICE, "hipEventCreate failed"));
    if (workspace) {
        if (ws_bytes < (int64_t)B->L.total)
            return bail(fail(MECH_E_NOMEM, "workspace of %lld bytes < %zu needed", (long long)ws_bytes, B->L.total));
        if (((uintptr_t)workspace & 255u) != 0)
            return bail(fail(MECH_E_INVALID, "workspace must be 256-byte aligned"));
        B->arena = (char*)workspace;
    } else {
        if (hipMalloc(&B->arena, B->L.total) != hipSuccess) {
            B->arena = nullptr;
            (void)hipGetLastError();
            return bail(fail(MECH_E_NOMEM, "hipMalloc of %zu bytes failed", B->L.total));
        }
        B->own_arena = true;
    }
    const Layout& L = B->L;
    double cd[64];
    float cf[64];
    for (int k = 0; k < 64; ++k) {
        cd[k] = params->c_adh[k];
        cf[k] = (float)params->c_adh[k];
    }
    if (hipMemcpy(B->arena + L.cadh, cd, sizeof cd, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(B->arena + L.cadh_f, cf, sizeof cf, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemsetAsync(B->arena + L.count, 0, (size_t)max_voxels * XSUB * 4, B->stream) != hipSuccess ||
        hipMemsetAsync(B->arena + L.stats, 0, STAT_SLOTS * 16, B->stream) != hipSuccess ||
        hipMemsetAsync(B->arena + L.start, 0, ((size_t)max_voxels * XSUB + 1) * 4, B->stream) != hipSuccess ||
        hipMemsetAsync(B->arena + L.hdr, 0, HDR_WORDS * 4, B->stream) != hipSuccess ||
        hipMemsetAsync(B->arena + L.split, 0, (N_XCD + 1) * 4, B->stream) != hipSuccess ||
        hipMemsetAsync(B->arena + L.work, 0, BAL_ENTRIES * 4, B->stream) != hipSuccess ||
        hipMemsetAsync(B->arena + L.slots, 0, (size_t)max_slots * sizeof(SlotDesc), B->stream) != hipSuccess)
        return bail(fail(MECH_E_DEVICE, "arena initialisation failed"));
    rc = sync_check(B);
    if (rc) return bail(rc);
    *out = B;
    return MECH_OK;
}

// Compacts the live slots to the front of the arena (drops retired ones), in their
// current order.  Runs on the batch stream; results are unchanged.
int repack(MechBatch* B)
{
    const Layout& L = B->L;
    const uint32_t n_old = B->n_cells;
    std::vector<int32_t> keep;
    uint32_t coff = 0, voff = 0;
    for (int32_t id : B->order) {
        HostSlot& s = B->slots[id];
        if (s.retired) {
            s.d.n_cells = 0;  // dropped by k_repack
        } else {
            s.d.prev_cell_off = s.d.cell_off;
            s.d.cell_off = coff;
            s.d.voxel_off = voff;
            coff += s.d.n_cells;
            voff += (uint32_t)s.d.nx * s.d.ny * s.d.nz;
            keep.push_back(id);
        }
        push_slot(B, id);
    }
    if (n_old > 0) {
        const int cur = B->parity, nxt = cur ^ 1;
        auto launch = [&](auto vpt_tag) {
            using VPT = decltype(vpt_tag);
            RepackArgs<VPT> a{};
            for (int c = 0; c < 3; ++c) {
                a.X[c] = B->at<double>(L.X[c]);
                a.XS[c] = B->at<double>(L.XS[c]);
                a.VP_cur[c] = B->at<VPT>(L.VP[cur][c]);
                a.VP_new[c] = B->at<VPT>(L.VP[nxt][c]);
            }
            a.R_cur = B->at<double>(L.R[cur]);
            a.R_new = B->at<double>(L.R[nxt]);
            a.T_cur = B->at<int32_t>(L.T[cur]);
            a.T_new = B->at<int32_t>(L.T[nxt]);
            a.ID_cur = B->at<uint32_t>(L.ID[cur]);
            a.ID_new = B->at<uint32_t>(L.ID[nxt]);
            a.slot_of = B->at<uint32_t>(L.slot_of);
            a.slot_new = B->at<uint32_t>(L.tmp_src);
            a.slots = B->at<SlotDesc>(L.slots);
            hipLaunchKernelGGL(k_repack<VPT>, dim3(blocks_for(n_old, BLOCK)), dim3(BLOCK), 0, B->stream, n_old, a);
        };
        if (is_fp32(B->prm))
            launch(float{});
        else
            launch(double{});
        if (coff > 0) {
            hipLaunchKernelGGL(k_copy_positions, dim3(blocks_for(coff, BLOCK)), dim3(BLOCK), 0, B->stream, coff,
                               B->at<double>(L.XS[0]), B->at<double>(L.XS[1]), B->at<double>(L.XS[2]),
                               B->at<double>(L.X[0]), B->at<double>(L.X[1]), B->at<double>(L.X[2]));
            hipLaunchKernelGGL(k_copy_u32, dim3(blocks_for(coff, BLOCK)), dim3(BLOCK), 0, B->stream, coff,
                               B->at<uint32_t>(L.tmp_src), B->at<uint32_t>(L.slot_of));
        }
        B->parity ^= 1;
    }
    for (int32_t id : B->order) {
        HostSlot& s = B->slots[id];
        if (s.retired) {
            s = HostSlot{s.d, false, false, false, 0, s.done, false};
            s.d = SlotDesc{};
            push_slot(B, id);
        }
    }
    B->order = keep;
    B->n_cells = coff;
    B->n_voxels = voff;
    push_header(B);
    HIP_TRY(hipGetLastError());
    return MECH_OK;
}

int admit_impl(MechBatch* B, const double lo[3], const double hi[3], int64_t n, const double* pos,
               const double* radius, const int32_t* type, const double* vprev, int64_t n_steps,
               int32_t* slot_out)
{
    int32_t dims[3];
    uint64_t V = 0;
    int rc = validate_domain(lo, hi, B->prm.voxel_size, dims, &V);
    if (rc) return rc;
    double rmax = 0.0;
    rc = validate_cells(&B->prm, lo, hi, n, pos, radius, type, vprev, &rmax);
    if (rc) return rc;
    auto free_id = [&]() {
        for (int32_t k = 0; k < B->cap_slots; ++k)
            if (!B->slots[k].used) return k;
        return -1;
    };
    int64_t live_c = 0, live_v = 0;
    bool any_retired = false;
    for (int32_t k : B->order) {
        if (B->slots[k].retired) {
            any_retired = true;
        } else {
            live_c += B->slots[k].d.n_cells;
            live_v += (int64_t)B->slots[k].d.nx * B->slots[k].d.ny * B->slots[k].d.nz;
        }
    }
    if (free_id() < 0 && !any_retired) return fail(MECH_E_FULL, "all %d slots are in use", B->cap_slots);
    if (live_c + n > B->cap_cells || live_v + (int64_t)V > B->cap_voxels)
        return fail(MECH_E_BUDGET, "request of %lld cells and %llu voxels does not fit (%lld/%lld cells, "
                    "%lld/%lld voxels in use)", (long long)n, (unsigned long long)V, (long long)live_c,
                    (long long)B->cap_cells, (long long)live_v, (long long)B->cap_voxels);
    // Retired slots hold their id and space until a compaction drops them.  Compact when
    // the new request needs the room or an id, or when retired cells or voxels outnumber
    // the live ones: every step still bins and moves the retired cells and scans their
    // voxels, so letting them pile up would slow the live simulations down.
    const int64_t dead_c = (int64_t)B->n_cells - live_c, dead_v = (int64_t)B->n_voxels - live_v;
    if (free_id() < 0 || (int64_t)B->n_cells + n > B->cap_cells ||
        (int64_t)B->n_voxels + (int64_t)V > B->cap_voxels ||
        (any_retired && (dead_c > live_c || dead_v > live_v))) {
        rc = repack(B);
        if (rc) return rc;
        // the compacted range may overlap cells that queued steps still write: the
        // copies below must come after them
        HIP_TRY(hipStreamSynchronize(B->stream));
    }
    const int32_t id = free_id();
    if (id < 0) return fail(MECH_E_FULL, "all %d slots are in use", B->cap_slots);
    HostSlot& s = B->slots[id];
    SlotDesc& d = s.d;
    d = slot_desc(B->prm, lo, hi, dims, rmax, n, n_steps, vprev != nullptr, B->n_cells, B->n_voxels);
    s.used = true;
    s.retired = false;
    s.reported = false;
    s.steps_total = n_steps;
    s.done_recorded = false;

    // the cells go to [cell_off, cell_off + n) of the current parity, in id order; the
    // copies run on the copy stream, so they overlap the steps already queued, which
    // do not touch this range
    const Layout& L = B->L;
    const size_t nn = (size_t)n;
    const size_t o = d.cell_off;
    std::vector<double> soa(3 * nn);
    std::vector<uint32_t> ids(nn), sl(nn, (uint32_t)id);
    std::vector<int32_t> tz;
    for (size_t i = 0; i < nn; ++i) {
        for (int c = 0; c < 3; ++c) soa[c * nn + i] = pos[3 * i + c];
        ids[i] = (uint32_t)(o + i);
    }
    const int p = B->parity;
    hipStream_t cs = B->copy_stream;
    int e = 0;
    auto H2D = [&](size_t off, const void* src, size_t bytes) {
        if (bytes && hipMemcpyAsync(B->arena + off, src, bytes, hipMemcpyHostToDevice, cs) != hipSuccess) e = 1;
    };
    for (int c = 0; c < 3; ++c) H2D(L.X[c] + o * 8, soa.data() + c * nn, nn * 8);
    H2D(L.R[p] + o * 8, radius, nn * 8);
    if (type) {
        H2D(L.T[p] + o * 4, type, nn * 4);
    } else {
        tz.assign(nn, 0);
        H2D(L.T[p] + o * 4, tz.data(), nn * 4);
    }
    H2D(L.ID[p] + o * 4, ids.data(), nn * 4);
    H2D(L.slot_of + o * 4, sl.data(), nn * 4);
    std::vector<double> vp64;
    std::vector<float> vp32;
    if (is_fp32(B->prm)) {
        vp32.assign(3 * nn, 0.f);
        if (vprev)
            for (size_t i = 0; i < nn; ++i)
                for (int c = 0; c < 3; ++c) vp32[c * nn + i] = (float)vprev[3 * i + c];
        for (int c = 0; c < 3; ++c) H2D(L.VP[p][c] + o * 4, vp32.data() + c * nn, nn * 4);
    } else {
        vp64.assign(3 * nn, 0.0);
        if (vprev)
            for (size_t i = 0; i < nn; ++i)
                for (int c = 0; c < 3; ++c) vp64[c * nn + i] = vprev[3 * i + c];
        for (int c = 0; c < 3; ++c) H2D(L.VP[p][c] + o * 8, vp64.data() + c * nn, nn * 8);
    }
    if (e) return fail(MECH_E_DEVICE, "host to device copy failed");
    // the host buffers above go out of scope: wait for the copy stream (only these copies)
    HIP_TRY(hipStreamSynchronize(cs));
    B->order.push_back(id);
    B->n_cells += (uint32_t)n;
    B->n_voxels += (uint32_t)V;
    push_slot(B, id);
    push_header(B);
    if (d.steps_left == 0) {  // nothing to run: complete at once
        HIP_TRY(hipEventRecord(s.done, B->stream));
        s.done_recorded = true;
    }
    HIP_TRY(hipGetLastError());
    if (slot_out) *slot_out = id;
    return MECH_OK;
}

// Host side of a step: parity, the host mirror of the device counters, and the event
// that marks the step at which a slot froze.
int after_step(MechBatch* B, bool gather)
{
    if (B->n_cells > 0) {
        if (gather) B->parity ^= 1;
        B->last_gather = gather;
    }
    ++B->reorder_phase;
    for (int32_t id : B->order) {
        HostSlot& s = B->slots[id];
        s.d.euler = 0;
        if (s.d.steps_left > 0 && --s.d.steps_left == 0 && !s.done_recorded) {
            HIP_TRY(hipEventRecord(s.done, B->stream));
            s.done_recorded = true;
        }
    }
    ++B->steps;
    return MECH_OK;
}

// A slot whose step counter reaches 0 within the next m steps: its completion event
// must be recorded after that very step, so such steps are launched one at a time.
bool slot_ends_within(const MechBatch* B, int m)
{
    for (int32_t id : B->order) {
        const int32_t left = B->slots[id].d.steps_left;
        if (left >= 1 && left <= m) return true;
    }
    return false;
}

int step_impl(MechBatch* B, int64_t n_steps)
{
    if (n_steps < 0) return fail(MECH_E_INVALID, "n_steps must be >= 0");
    HIP_TRY(hipSetDevice(B->device));
    const bool eager = (B->prm.flags & MECH_FLAG_NO_GRAPH) != 0;
    for (int64_t k = 0; k < n_steps; ++k) {
        if (!eager && B->reorder_every == 1 && B->n_cells > 0 && n_steps - k >= RUN_STEPS &&
            !slot_ends_within(B, RUN_STEPS - 1)) {
            if (!B->graphs_ready) {
                int rc = build_graphs(B);
                if (rc) return rc;
            }
            HIP_TRY(hipGraphLaunch(B->gexec_run[B->parity], B->stream));
            HIP_TRY(hipGetLastError());
            for (int i = 0; i < RUN_STEPS; ++i) {
                int rc = after_step(B, true);
                if (rc) return rc;
            }
            k += RUN_STEPS - 1;
            continue;
        }
        const bool gather = gather_now(B);
        if (B->n_cells > 0) {
            if (eager) {
                enqueue_step(B, B->parity, gather);
            } else {
                if (!B->graphs_ready) {
                    int rc = build_graphs(B);
                    if (rc) return rc;
                }
                HIP_TRY(hipGraphLaunch(gather ? B->gexec[B->parity] : B->gexec_inplace[B->parity], B->stream));
            }
        } else {
            enqueue_step_end(B);  // keeps the device step counters in line with the host's
        }
        HIP_TRY(hipGetLastError());
        int rc = after_step(B, gather);
        if (rc) return rc;
    }
    return MECH_OK;
}

int read_slot(MechBatch* B, int32_t id, double* pos, double* vel, int64_t n_cells)
{
    if (id < 0 || id >= B->cap_slots || !B->slots[id].used || B->slots[id].retired)
        return fail(MECH_E_INVALID, "slot %d holds no simulation", id);
    const SlotDesc& d = B->slots[id].d;
    if (!pos) return fail(MECH_E_INVALID, "pos is NULL");
    if (n_cells != (int64_t)d.n_cells)
        return fail(MECH_E_INVALID, "n_cells %lld != slot size %u", (long long)n_cells, d.n_cells);
    HIP_TRY(hipSetDevice(B->device));
    if (d.n_cells == 0) return MECH_OK;
    const Layout& L = B->L;
    const int p = B->parity;
    const uint32_t n = d.n_cells;
    double* st = B->at<double>(L.stage);
    if (is_fp32(B->prm))
        hipLaunchKernelGGL(k_unpermute<float>, dim3(blocks_for(n, BLOCK)), dim3(BLOCK), 0, B->stream, d.cell_off, n,
                           B->at<uint32_t>(L.ID[p]), B->at<double>(L.X[0]), B->at<double>(L.X[1]),
                           B->at<double>(L.X[2]), B->at<float>(L.VP[p][0]), B->at<float>(L.VP[p][1]),
                           B->at<float>(L.VP[p][2]), st, st + 3 * (size_t)n);
    else
        hipLaunchKernelGGL(k_unpermute<double>, dim3(blocks_for(n, BLOCK)), dim3(BLOCK), 0, B->stream, d.cell_off, n,
                           B->at<uint32_t>(L.ID[p]), B->at<double>(L.X[0]), B->at<double>(L.X[1]),
                           B->at<double>(L.X[2]), B->at<double>(L.VP[p][0]), B->at<double>(L.VP[p][1]),
                           B->at<double>(L.VP[p][2]), st, st + 3 * (size_t)n);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(pos, st, 24 * (size_t)n, hipMemcpyDeviceToHost, B->stream));
    if (vel) HIP_TRY(hipMemcpyAsync(vel, st + 3 * (size_t)n, 24 * (size_t)n, hipMemcpyDeviceToHost, B->stream));
    int rc = sync_check(B);
    if (rc) return rc;
    for (size_t i = 0; i < 3 * (size_t)n; ++i)
        if (!std::isfinite(pos[i]) || (vel && !std::isfinite(vel[i])))
            return fail(MECH_E_NONFINITE, "state holds a non-finite value at cell %zu", i / 3);
    return MECH_OK;
}

int stats_impl(MechBatch* B, int64_t* steps, int64_t* interactions, int64_t* candidates)
{
    HIP_TRY(hipSetDevice(B->device));
    int rc = sync_check(B);
    if (rc) return rc;
    std::vector<unsigned long long> slots(2 * STAT_SLOTS);
    HIP_TRY(hipMemcpy(slots.data(), B->arena + B->L.stats, slots.size() * 8, hipMemcpyDeviceToHost));
    unsigned long long st[2] = {0, 0};
    for (uint32_t k = 0; k < STAT_SLOTS; ++k) {
        st[0] += slots[2 * k];
        st[1] += slots[2 * k + 1];
    }
    if (steps) *steps = B->steps;
    if (interactions) *interactions = (int64_t)st[0];
    if (candidates) *candidates = (int64_t)st[1];
    return MECH_OK;
}

int profile_impl(MechBatch* B, int64_t n_steps, double* phase_ms)
{
    if (!phase_ms || n_steps < 1) return fail(MECH_E_INVALID, "need phase_ms and n_steps >= 1");
    HIP_TRY(hipSetDevice(B->device));
    phase_ms[0] = phase_ms[1] = 0.0;
    if (B->n_cells == 0) return step_impl(B, n_steps);
    hipEvent_t ev[3];
    for (int k = 0; k < 3; ++k) HIP_TRY(hipEventCreate(&ev[k]));
    double acc[2] = {0.0, 0.0};
    int rc = MECH_OK;
    for (int64_t s = 0; s < n_steps && rc == MECH_OK; ++s) {
        const int p = B->parity;
        const bool gather = gather_now(B);
        (void)hipEventRecord(ev[0], B->stream);
        B->step_start = true;
        if (gather)
            enqueue_binning_any(B);
        else
            enqueue_binning_inplace(B);
        B->step_start = false;
        (void)hipEventRecord(ev[1], B->stream);
        if (gather)
            enqueue_force_any(B, p ^ 1);
        else
            enqueue_force_inplace_any(B);
        (void)hipEventRecord(ev[2], B->stream);
        enqueue_division(B, gather ? p ^ 1 : p);
        enqueue_death(B, gather ? p ^ 1 : p);
        rc = after_step(B, gather);
        if (rc == MECH_OK) rc = sync_check(B);
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

// The largest arena within a byte budget: cells and voxels = ceil(voxels_per_cell * cells)
// (at least one), found by bisection over the layout's exact size.
int budget_capacity(const MechParams* params, int64_t budget, double vpc, int32_t max_slots, int64_t* cells_out,
                    int64_t* voxels_out)
{
    int rc = validate_physics(params);
    if (rc) return rc;
    if (!(std::isfinite(vpc) && vpc > 0.0 && vpc <= 1e6))
        return fail(MECH_E_INVALID, "voxels_per_cell must be in (0, 1e6]");
    if (max_slots < 1 || max_slots > 65536) return fail(MECH_E_INVALID, "max_slots out of range");
    const int64_t vmax = (int64_t(1) << 30) - 1;
    auto voxels_for = [&](int64_t c) { return std::min<int64_t>(vmax, std::max<int64_t>(1, (int64_t)std::ceil(vpc * (double)c))); };
    auto bytes = [&](int64_t c) { return (int64_t)make_layout(*params, c, (uint64_t)voxels_for(c), max_slots).total; };
    if (budget < bytes(1)) return fail(MECH_E_BUDGET, "a budget of %lld bytes holds no cell (%lld needed for one)",
                                       (long long)budget, (long long)bytes(1));
    int64_t lo = 1, hi = std::min<int64_t>((int64_t(1) << 31) - 1, (int64_t)((double)vmax / vpc));
    hi = std::max<int64_t>(hi, 1);
    if (bytes(hi) <= budget) lo = hi;
    while (lo < hi) {   // bytes(lo) <= budget < bytes(hi + 1) after the loop
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (bytes(mid) <= budget) lo = mid; else hi = mid - 1;
    }
    *cells_out = lo;
    *voxels_out = voxels_for(lo);
    return MECH_OK;
}

int64_t batch_bytes(const MechParams* params, int64_t max_cells, int64_t max_voxels, int32_t max_slots)
{
    int rc = validate_physics(params);
    if (rc) return rc;
    if (max_cells < 0 || max_cells >= (int64_t(1) << 31) || max_voxels < 1 || max_voxels >= (int64_t(1) << 30) ||
        max_slots < 1)
        return fail(MECH_E_INVALID, "bad capacity");
    return (int64_t)make_layout(*params, max_cells, (uint64_t)max_voxels, max_slots).total;
}

}  // namespace

// ------------------------------------------------------------------------ C ABI

namespace {

// Device address of the static scratch on the current device, looked up once per device
// (each device holds its own copy of the array at its own address).
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

int noalloc_scratch(int device, void** out)
{
    if (device < 0 || device >= MAX_DEVICES) return fail(MECH_E_DEVICE, "device %d out of range", device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MECH_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return MECH_OK;
}

// create_population + step_mechanics + read_state with every device array in the static
// scratch: the same layout, the same kernels in the same order (direct launches), no
// allocation, no stream, event or graph.
int noalloc_impl(const MechParams* params, int64_t n, const double* pos, const double* radius, const int32_t* type,
                 const double* vprev, int64_t n_steps, void* hip_stream, double* pos_out, double* vel_out,
                 int64_t* interactions)
{
    int rc = validate_physics(params);
    if (rc) return rc;
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(MECH_E_INVALID, "n_cells out of range");
    if (n_steps < 0) return fail(MECH_E_INVALID, "n_steps must be >= 0");
    if (n > 0 && !pos_out) return fail(MECH_E_INVALID, "pos_out is NULL");
    int32_t dims[3];
    uint64_t V = 0;
    rc = validate_domain(params->domain_lo, params->domain_hi, params->voxel_size, dims, &V);
    if (rc) return rc;
    double rmax = 0.0;
    rc = validate_cells(params, params->domain_lo, params->domain_hi, n, pos, radius, type, vprev, &rmax);
    if (rc) return rc;
    MechBatch B;   // on the stack: its vectors stay empty (no slot bookkeeping here)
    B.prm = *params;
    B.phys = phys_args(*params);
    B.cap_cells = n;
    B.cap_voxels = (int64_t)V;
    B.cap_slots = 1;
    B.L = make_layout(*params, n, V, 1);
    if (B.L.total > (size_t)MECH_NOALLOC_SCRATCH_BYTES)
        return fail(MECH_E_NOMEM, "%lld cells and %llu voxels need %zu bytes, the static scratch holds %llu",
                    (long long)n, (unsigned long long)V, B.L.total, (unsigned long long)MECH_NOALLOC_SCRATCH_BYTES);
    HIP_TRY(hipGetDevice(&B.device));
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, B.device) != hipSuccess || cus < 1)
            cus = 256;
        B.cus = cus;
    }
    void* base = nullptr;
    rc = noalloc_scratch(B.device, &base);
    if (rc) return rc;
    B.arena = (char*)base;
    B.stream = (hipStream_t)hip_stream;
    const Layout& L = B.L;
    const hipStream_t st = B.stream;
    // the scratch keeps the last call's contents: everything read before it is written
    // is set here (adhesion tables, counts, starts, counters, header, slot table)
    double cd[64];
    float cf[64];
    for (int k = 0; k < 64; ++k) {
        cd[k] = params->c_adh[k];
        cf[k] = (float)params->c_adh[k];
    }
    HIP_TRY(hipMemcpyAsync(B.arena + L.cadh, cd, sizeof cd, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(B.arena + L.cadh_f, cf, sizeof cf, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemsetAsync(B.arena + L.count, 0, (size_t)V * XSUB * 4, st));
    HIP_TRY(hipMemsetAsync(B.arena + L.start, 0, ((size_t)V * XSUB + 1) * 4, st));
    HIP_TRY(hipMemsetAsync(B.arena + L.stats, 0, STAT_SLOTS * 16, st));
    HIP_TRY(hipMemsetAsync(B.arena + L.hdr, 0, HDR_WORDS * 4, st));
    HIP_TRY(hipMemsetAsync(B.arena + L.split, 0, (N_XCD + 1) * 4, st));
    HIP_TRY(hipMemsetAsync(B.arena + L.work, 0, BAL_ENTRIES * 4, st));
    const SlotDesc d = slot_desc(*params, params->domain_lo, params->domain_hi, dims, rmax, n, -1, vprev != nullptr,
                                 0u, 0u);
    hipLaunchKernelGGL(k_set_slot, dim3(1), dim3(1), 0, st, B.at<SlotDesc>(L.slots), 0u, d);
    B.n_cells = (uint32_t)n;
    B.n_voxels = (uint32_t)V;
    push_header(&B);
    if (n > 0) {
        const uint32_t nu = (uint32_t)n;
        double* stage = B.at<double>(L.stage);
        HIP_TRY(hipMemcpyAsync(stage, pos, 24 * (size_t)n, hipMemcpyHostToDevice, st));
        if (vprev) HIP_TRY(hipMemcpyAsync(stage + 3 * (size_t)n, vprev, 24 * (size_t)n, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(B.arena + L.R[0], radius, 8 * (size_t)n, hipMemcpyHostToDevice, st));
        if (type)
            HIP_TRY(hipMemcpyAsync(B.arena + L.T[0], type, 4 * (size_t)n, hipMemcpyHostToDevice, st));
        else
            HIP_TRY(hipMemsetAsync(B.arena + L.T[0], 0, 4 * (size_t)n, st));
        if (is_fp32(B.prm))
            hipLaunchKernelGGL(k_load_cells<float>, dim3(blocks_for(nu, BLOCK)), dim3(BLOCK), 0, st, nu, stage,
                               vprev != nullptr, B.at<double>(L.X[0]), B.at<double>(L.X[1]), B.at<double>(L.X[2]),
                               B.at<uint32_t>(L.ID[0]), B.at<uint32_t>(L.slot_of), B.at<float>(L.VP[0][0]),
                               B.at<float>(L.VP[0][1]), B.at<float>(L.VP[0][2]));
        else
            hipLaunchKernelGGL(k_load_cells<double>, dim3(blocks_for(nu, BLOCK)), dim3(BLOCK), 0, st, nu, stage,
                               vprev != nullptr, B.at<double>(L.X[0]), B.at<double>(L.X[1]), B.at<double>(L.X[2]),
                               B.at<uint32_t>(L.ID[0]), B.at<uint32_t>(L.slot_of), B.at<double>(L.VP[0][0]),
                               B.at<double>(L.VP[0][1]), B.at<double>(L.VP[0][2]));
        HIP_TRY(hipGetLastError());
        // the initial binning of create_population
        enqueue_binning_any(&B);
        hipLaunchKernelGGL(k_copy_positions, dim3(blocks_for(nu, BLOCK)), dim3(BLOCK), 0, st, nu,
                           B.at<double>(L.XS[0]), B.at<double>(L.XS[1]), B.at<double>(L.XS[2]),
                           B.at<double>(L.X[0]), B.at<double>(L.X[1]), B.at<double>(L.X[2]));
        B.parity ^= 1;
        for (int64_t k = 0; k < n_steps; ++k) {
            enqueue_step(&B, B.parity, true);
            B.parity ^= 1;
        }
        HIP_TRY(hipGetLastError());
        // read_state: un-permute into the staging area, then to the caller
        const int p = B.parity;
        if (is_fp32(B.prm))
            hipLaunchKernelGGL(k_unpermute<float>, dim3(blocks_for(nu, BLOCK)), dim3(BLOCK), 0, st, 0u, nu,
                               B.at<uint32_t>(L.ID[p]), B.at<double>(L.X[0]), B.at<double>(L.X[1]),
                               B.at<double>(L.X[2]), B.at<float>(L.VP[p][0]), B.at<float>(L.VP[p][1]),
                               B.at<float>(L.VP[p][2]), stage, stage + 3 * (size_t)n);
        else
            hipLaunchKernelGGL(k_unpermute<double>, dim3(blocks_for(nu, BLOCK)), dim3(BLOCK), 0, st, 0u, nu,
                               B.at<uint32_t>(L.ID[p]), B.at<double>(L.X[0]), B.at<double>(L.X[1]),
                               B.at<double>(L.X[2]), B.at<double>(L.VP[p][0]), B.at<double>(L.VP[p][1]),
                               B.at<double>(L.VP[p][2]), stage, stage + 3 * (size_t)n);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(pos_out, stage, 24 * (size_t)n, hipMemcpyDeviceToHost, st));
        if (vel_out) HIP_TRY(hipMemcpyAsync(vel_out, stage + 3 * (size_t)n, 24 * (size_t)n, hipMemcpyDeviceToHost, st));
    }
    unsigned long long stat[2 * STAT_SLOTS];
    if (interactions) HIP_TRY(hipMemcpyAsync(stat, B.arena + L.stats, sizeof stat, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipGetLastError());
    if (interactions) {
        unsigned long long sum = 0;
        for (uint32_t k = 0; k < STAT_SLOTS; ++k) sum += stat[2 * k];
        *interactions = (int64_t)sum;
    }
    for (size_t i = 0; i < 3 * (size_t)n; ++i)
        if (!std::isfinite(pos_out[i]) || (vel_out && !std::isfinite(vel_out[i])))
            return fail(MECH_E_NONFINITE, "state holds a non-finite value at cell %zu", i / 3);
    return MECH_OK;
}

}  // namespace

// The library's other source files (the microenvironment solver) report their errors
// through the same thread-local text; not exported.
__attribute__((visibility("hidden"))) int mech_report_error(int code, const char* text)
{
    g_err = text;
    return code;
}

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

// ---- single population (a batch of one slot)

int64_t population_workspace_bytes(const MechParams* params, int64_t n_cells)
{
    int rc = validate_physics(params);
    if (rc) return rc;
    if (n_cells < 0 || n_cells >= (int64_t(1) << 31)) return fail(MECH_E_INVALID, "n_cells out of range");
    int32_t dims[3];
    uint64_t V = 0;
    rc = validate_domain(params->domain_lo, params->domain_hi, params->voxel_size, dims, &V);
    if (rc) return rc;
    return batch_bytes(params, n_cells, (int64_t)V, 1);
}

static int create_pop_impl(const MechParams* params, int64_t n_cells, const double* pos, const double* radius,
                           const int32_t* type, const double* prev_velocity, void* hip_stream, void* workspace,
                           int64_t ws_bytes, MechPopulation** out, int64_t max_cells = -1)
{
    if (!out) return fail(MECH_E_INVALID, "out is NULL");
    *out = nullptr;
    int rc = validate_physics(params);
    if (rc) return rc;
    int32_t dims[3];
    uint64_t V = 0;
    rc = validate_domain(params->domain_lo, params->domain_hi, params->voxel_size, dims, &V);
    if (rc) return rc;
    double rmax = 0.0;
    rc = validate_cells(params, params->domain_lo, params->domain_hi, n_cells, pos, radius, type,
                        prev_velocity, &rmax);
    if (rc) return rc;
    if (max_cells < 0) max_cells = n_cells;
    if (max_cells < n_cells || max_cells >= (int64_t(1) << 31))
        return fail(MECH_E_INVALID, "max_cells %lld out of range", (long long)max_cells);
    MechBatch* B = nullptr;
    rc = create_batch_impl(params, max_cells, (int64_t)V, 1, hip_stream, workspace, ws_bytes, &B);
    if (rc) return rc;
    int32_t slot = -1;
    rc = admit_impl(B, params->domain_lo, params->domain_hi, n_cells, pos, radius, type, prev_velocity, -1, &slot);
    if (rc) {
        release(B);
        return rc;
    }
    // initial binning, so that read_binning describes the given positions
    if (n_cells > 0) {
        enqueue_binning_any(B);
        const Layout& L = B->L;
        hipLaunchKernelGGL(k_copy_positions, dim3(blocks_for(n_cells, BLOCK)), dim3(BLOCK), 0, B->stream,
                           (uint32_t)n_cells, B->at<double>(L.XS[0]), B->at<double>(L.XS[1]),
                           B->at<double>(L.XS[2]), B->at<double>(L.X[0]), B->at<double>(L.X[1]),
                           B->at<double>(L.X[2]));
        B->parity ^= 1;
    }
    rc = sync_check(B);
    if (rc) {
        release(B);
        return rc;
    }
    MechPopulation* P = new MechPopulation();
    P->b = B;
    P->n = n_cells;
    *out = P;
    return MECH_OK;
}

int create_population(const MechParams* params, int64_t n_cells, const double* pos, const double* radius,
                      const int32_t* type, const double* prev_velocity, void* hip_stream, MechPopulation** out)
{
    return create_pop_impl(params, n_cells, pos, radius, type, prev_velocity, hip_stream, nullptr, 0, out);
}

int create_population_cap(const MechParams* params, int64_t n_cells, int64_t max_cells, const double* pos,
                          const double* radius, const int32_t* type, const double* prev_velocity, void* hip_stream,
                          MechPopulation** out)
{
    return create_pop_impl(params, n_cells, pos, radius, type, prev_velocity, hip_stream, nullptr, 0, out,
                           max_cells);
}

int create_population_in(const MechParams* params, int64_t n_cells, const double* pos, const double* radius,
                         const int32_t* type, const double* prev_velocity, void* hip_stream, void* workspace,
                         int64_t workspace_bytes, MechPopulation** out)
{
    if (!workspace) {
        if (out) *out = nullptr;
        return fail(MECH_E_INVALID, "workspace is NULL");
    }
    return create_pop_impl(params, n_cells, pos, radius, type, prev_velocity, hip_stream, workspace,
                           workspace_bytes, out);
}

int step_mechanics_noalloc(const MechParams* params, int64_t n_cells, const double* pos, const double* radius,
                           const int32_t* type, const double* prev_velocity, int64_t n_steps, void* hip_stream,
                           double* pos_out, double* vel_out, int64_t* interactions)
{
    return noalloc_impl(params, n_cells, pos, radius, type, prev_velocity, n_steps, hip_stream, pos_out, vel_out,
                        interactions);
}

int step_mechanics(MechPopulation* P, int64_t n_steps)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    return step_impl(P->b, n_steps);
}

int profile_step(MechPopulation* P, int64_t n_steps, double* phase_ms)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    return profile_impl(P->b, n_steps, phase_ms);
}

static int refresh_size(MechPopulation* P);

int read_state(MechPopulation* P, double* pos, double* vel, int64_t n_cells)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    if (!pos) return fail(MECH_E_INVALID, "pos is NULL");
    int rc = refresh_size(P);
    if (rc) return rc;
    if (n_cells != P->n) return fail(MECH_E_INVALID, "n_cells %lld != population size %lld", (long long)n_cells, (long long)P->n);
    return read_slot(P->b, 0, pos, vel, n_cells);
}

int read_binning(MechPopulation* P, uint32_t* voxel_of_cell, uint32_t* voxel_start, uint32_t* sorted_ids,
                 uint32_t* occ, int64_t* n_occ, int64_t* n_voxels)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    int rc = refresh_size(P);
    if (rc) return rc;
    MechBatch* B = P->b;
    HIP_TRY(hipSetDevice(B->device));
    rc = sync_check(B);
    if (rc) return rc;
    const Layout& L = B->L;
    const size_t n = (size_t)P->n;
    const size_t V = (size_t)B->n_voxels;
    if (n_voxels) *n_voxels = (int64_t)V;
    uint32_t m = 0;
    if (n > 0) HIP_TRY(hipMemcpy(&m, B->arena + L.hdr + 4 * H_OCC, 4, hipMemcpyDeviceToHost));
    if (n_occ) *n_occ = m;
    if (voxel_start) {
        // voxel v starts at its first bin, XSUB * v (one contiguous copy: a strided copy
        // of tens of millions of 4-byte rows is far slower)
        if (n > 0) {
            std::vector<uint32_t> bins(XSUB * V + 1);
            HIP_TRY(hipMemcpy(bins.data(), B->arena + L.start, bins.size() * 4, hipMemcpyDeviceToHost));
            for (size_t v = 0; v <= V; ++v) voxel_start[v] = bins[XSUB * v];
        } else {
            std::memset(voxel_start, 0, (V + 1) * 4);
        }
    }
    if (occ && m) HIP_TRY(hipMemcpy(occ, B->arena + L.occ, (size_t)m * 4, hipMemcpyDeviceToHost));
    if (n == 0) return MECH_OK;
    if (!B->last_gather) {
        // cells left in place: storage order is not the sorted order; perm maps one to
        // the other
        std::vector<uint32_t> perm(n), ids(n), vc(n);
        HIP_TRY(hipMemcpy(perm.data(), B->arena + L.off, n * 4, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(ids.data(), B->arena + L.ID[B->parity], n * 4, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(vc.data(), B->arena + L.vid_cur, n * 4, hipMemcpyDeviceToHost));
        if (sorted_ids)
            for (size_t q = 0; q < n; ++q) sorted_ids[q] = ids[perm[q]];
        if (voxel_of_cell)
            for (size_t q = 0; q < n; ++q) voxel_of_cell[ids[q]] = vc[q] / XSUB;
        return MECH_OK;
    }
    std::vector<uint32_t> ids(n), vs(n);
    HIP_TRY(hipMemcpy(ids.data(), B->arena + L.ID[B->parity], n * 4, hipMemcpyDeviceToHost));
    if (sorted_ids) std::memcpy(sorted_ids, ids.data(), n * 4);
    if (voxel_of_cell) {
        HIP_TRY(hipMemcpy(vs.data(), B->arena + L.vid_sorted, n * 4, hipMemcpyDeviceToHost));
        for (size_t s = 0; s < n; ++s) voxel_of_cell[ids[s]] = vs[s] / XSUB;
    }
    return MECH_OK;
}

int read_stats(MechPopulation* P, int64_t* steps, int64_t* interactions, int64_t* candidates)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    return stats_impl(P->b, steps, interactions, candidates);
}

int read_xcd_split(MechPopulation* P, uint32_t* split)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    if (!split) return fail(MECH_E_INVALID, "split is NULL");
    MechBatch* B = P->b;
    HIP_TRY(hipSetDevice(B->device));
    const int rc = sync_check(B);
    if (rc) return rc;
    HIP_TRY(hipMemcpy(split, B->arena + B->L.split, (N_XCD + 1) * 4, hipMemcpyDeviceToHost));
    return MECH_OK;
}

int population_set_reorder(MechPopulation* P, int32_t every)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    if (every < 0) return fail(MECH_E_INVALID, "every must be >= 0");
    MechBatch* B = P->b;
    HIP_TRY(hipSetDevice(B->device));
    HIP_TRY(hipStreamSynchronize(B->stream));
    drop_graphs(B);
    if (every == 0 && B->n_cells > 0) {
        // back to the order the cells were given in, then binned where they are
        const Layout& L = B->L;
        const int cur = B->parity, nxt = cur ^ 1;
        const uint32_t nbc = cell_grid(B);
        const uint32_t* hdr = B->at<uint32_t>(L.hdr);
        auto order = [&](auto tag) {
            using VPT = decltype(tag);
            OrderArgs<VPT> o{};
            for (int c = 0; c < 3; ++c) {
                o.X[c] = B->at<double>(L.X[c]);
                o.XS[c] = B->at<double>(L.XS[c]);
                o.VP_cur[c] = B->at<VPT>(L.VP[cur][c]);
                o.VP_new[c] = B->at<VPT>(L.VP[nxt][c]);
            }
            o.R_cur = B->at<double>(L.R[cur]);
            o.R_new = B->at<double>(L.R[nxt]);
            o.T_cur = B->at<int32_t>(L.T[cur]);
            o.T_new = B->at<int32_t>(L.T[nxt]);
            o.ID_cur = B->at<uint32_t>(L.ID[cur]);
            o.ID_new = B->at<uint32_t>(L.ID[nxt]);
            hipLaunchKernelGGL(k_order_by_id<VPT>, dim3(nbc), dim3(BLOCK), 0, B->stream, hdr, o);
        };
        if (is_fp32(B->prm))
            order(float{});
        else
            order(double{});
        hipLaunchKernelGGL(k_commit, dim3(nbc), dim3(BLOCK), 0, B->stream, hdr, B->at<double>(L.XS[0]),
                           B->at<double>(L.XS[1]), B->at<double>(L.XS[2]), B->at<double>(L.X[0]),
                           B->at<double>(L.X[1]), B->at<double>(L.X[2]));
        B->parity = nxt;
        enqueue_binning_inplace(B);
        B->last_gather = false;
        int rc = sync_check(B);
        if (rc) return rc;
    }
    B->reorder_every = every;
    B->reorder_phase = 0;
    return MECH_OK;
}

int population_get_tuning(MechPopulation* P, MechTuning* out)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    return batch_get_tuning(P->b, out);
}

int population_set_tuning(MechPopulation* P, const MechTuning* t)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    return batch_set_tuning(P->b, t);
}

// A growing population's size lives on the device: wait and copy it to the host mirrors.
static int refresh_size(MechPopulation* P)
{
    MechBatch* B = P->b;
    if (!B->growing) return MECH_OK;
    HIP_TRY(hipSetDevice(B->device));
    int rc = sync_check(B);
    if (rc) return rc;
    uint32_t n = 0;
    HIP_TRY(hipMemcpy(&n, B->arena + B->L.hdr + 4 * H_CELLS, 4, hipMemcpyDeviceToHost));
    P->n = n;
    B->n_cells = n;
    B->slots[0].d.n_cells = n;
    return MECH_OK;
}

int population_size(MechPopulation* P, int64_t* n_cells)
{
    if (!P || !n_cells) return fail(MECH_E_INVALID, "population or n_cells is NULL");
    int rc = refresh_size(P);
    if (rc) return rc;
    *n_cells = P->n;
    return MECH_OK;
}

int population_set_division(MechPopulation* P, double p_div, uint64_t seed)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    if (!(p_div >= 0.0 && p_div <= 1.0)) return fail(MECH_E_INVALID, "p_div must lie in [0, 1]");
    MechBatch* B = P->b;
    if (B->cap_slots != 1) return fail(MECH_E_INVALID, "division needs a population");
    HIP_TRY(hipSetDevice(B->device));
    HIP_TRY(hipStreamSynchronize(B->stream));
    drop_graphs(B);
    B->p_div = p_div;
    B->div_seed = seed;
    if (p_div > 0.0) B->growing = true;
    return MECH_OK;
}

int population_set_death(MechPopulation* P, double p_death)
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    if (!(p_death >= 0.0 && p_death <= 1.0)) return fail(MECH_E_INVALID, "p_death must lie in [0, 1]");
    MechBatch* B = P->b;
    if (B->cap_slots != 1) return fail(MECH_E_INVALID, "death needs a population");
    HIP_TRY(hipSetDevice(B->device));
    HIP_TRY(hipStreamSynchronize(B->stream));
    drop_graphs(B);
    B->p_death = p_death;
    if (p_death > 0.0) B->growing = true;
    return MECH_OK;
}

int population_info(MechPopulation* P, int64_t* n_cells, int32_t dims[3])
{
    if (!P) return fail(MECH_E_INVALID, "population is NULL");
    int rc = refresh_size(P);
    if (rc) return rc;
    if (n_cells) *n_cells = P->n;
    if (dims) {
        const SlotDesc& d = P->b->slots[0].d;
        dims[0] = d.nx;
        dims[1] = d.ny;
        dims[2] = d.nz;
    }
    return MECH_OK;
}

void* population_stream(MechPopulation* P) { return P ? (void*)P->b->stream : nullptr; }

int destroy_population(MechPopulation* P)
{
    if (!P) return MECH_OK;
    MechBatch* B = P->b;
    (void)hipSetDevice(B->device);
    hipError_t e = B->stream ? hipStreamSynchronize(B->stream) : hipSuccess;
    release(B);
    delete P;
    if (e != hipSuccess) return fail(MECH_E_DEVICE, "stream error at destroy: %s", hipGetErrorString(e));
    return MECH_OK;
}

// ---- batches of independent simulations

int64_t batch_workspace_bytes(const MechParams* params, int64_t max_cells, int64_t max_voxels, int32_t max_slots)
{
    return batch_bytes(params, max_cells, max_voxels, max_slots);
}

int64_t batch_request_voxels(const MechParams* params, const double domain_lo[3], const double domain_hi[3])
{
    int rc = validate_physics(params);
    if (rc) return rc;
    int32_t dims[3];
    uint64_t V = 0;
    rc = validate_domain(domain_lo, domain_hi, params->voxel_size, dims, &V);
    if (rc) return rc;
    return (int64_t)V;
}

int create_batch(const MechParams* params, int64_t max_cells, int64_t max_voxels, int32_t max_slots,
                 void* hip_stream, MechBatch** out)
{
    return create_batch_impl(params, max_cells, max_voxels, max_slots, hip_stream, nullptr, 0, out);
}

int create_batch_in(const MechParams* params, int64_t max_cells, int64_t max_voxels, int32_t max_slots,
                    void* hip_stream, void* workspace, int64_t workspace_bytes, MechBatch** out)
{
    if (!workspace) {
        if (out) *out = nullptr;
        return fail(MECH_E_INVALID, "workspace is NULL");
    }
    return create_batch_impl(params, max_cells, max_voxels, max_slots, hip_stream, workspace, workspace_bytes, out);
}

int batch_budget_capacity(const MechParams* params, int64_t hbm_budget_bytes, double voxels_per_cell,
                          int32_t max_slots, int64_t* max_cells, int64_t* max_voxels)
{
    if (!max_cells || !max_voxels) return fail(MECH_E_INVALID, "max_cells or max_voxels is NULL");
    return budget_capacity(params, hbm_budget_bytes, voxels_per_cell, max_slots, max_cells, max_voxels);
}

int create_batch_budget(const MechParams* params, int64_t hbm_budget_bytes, double voxels_per_cell,
                        int32_t max_slots, void* hip_stream, MechBatch** out)
{
    if (out) *out = nullptr;
    int64_t cells = 0, voxels = 0;
    int rc = budget_capacity(params, hbm_budget_bytes, voxels_per_cell, max_slots, &cells, &voxels);
    if (rc) return rc;
    return create_batch_impl(params, cells, voxels, max_slots, hip_stream, nullptr, 0, out);
}

int batch_capacity(MechBatch* B, int64_t* max_cells, int64_t* max_voxels, int32_t* max_slots,
                   int64_t* arena_bytes)
{
    if (!B) return fail(MECH_E_INVALID, "batch is NULL");
    if (max_cells) *max_cells = B->cap_cells;
    if (max_voxels) *max_voxels = B->cap_voxels;
    if (max_slots) *max_slots = B->cap_slots;
    if (arena_bytes) *arena_bytes = (int64_t)B->L.total;
    return MECH_OK;
}

int batch_mark_clock(MechBatch* B)
{
    if (!B) return fail(MECH_E_INVALID, "batch is NULL");
    HIP_TRY(hipSetDevice(B->device));
    HIP_TRY(hipEventRecord(B->clock, B->stream));
    HIP_TRY(hipEventSynchronize(B->clock));
    B->clock_marked = true;
    return MECH_OK;
}

int batch_slot_done_ms(MechBatch* B, int32_t slot, double* ms)
{
    if (!B || !ms) return fail(MECH_E_INVALID, "batch or ms is NULL");
    if (slot < 0 || slot >= B->cap_slots || !B->slots[(size_t)slot].used)
        return fail(MECH_E_INVALID, "slot %d holds no simulation", slot);
    const HostSlot& s = B->slots[(size_t)slot];
    if (!B->clock_marked) return fail(MECH_E_INVALID, "batch_mark_clock was not called");
    if (!s.done_recorded) return fail(MECH_E_INVALID, "slot %d has not finished its steps", slot);
    HIP_TRY(hipSetDevice(B->device));
    const hipError_t q = hipEventQuery(s.done);
    if (q == hipErrorNotReady) return fail(MECH_E_INVALID, "slot %d has not finished on the device yet", slot);
    if (q != hipSuccess) return fail(MECH_E_DEVICE, "hipEventQuery failed: %s", hipGetErrorString(q));
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, B->clock, s.done));
    *ms = (double)t;
    return MECH_OK;
}

int batch_admit(MechBatch* B, const double domain_lo[3], const double domain_hi[3], int64_t n_cells,
                const double* pos, const double* radius, const int32_t* type, const double* prev_velocity,
                int64_t n_steps, int32_t* slot_out)
{
    if (!B) return fail(MECH_E_INVALID, "batch is NULL");
    if (!domain_lo || !domain_hi) return fail(MECH_E_INVALID, "domain is NULL");
    HIP_TRY(hipSetDevice(B->device));
    return admit_impl(B, domain_lo, domain_hi, n_cells, pos, radius, type, prev_velocity, n_steps, slot_out);
}

int batch_step(MechBatch* B, int64_t n_steps)
{
    if (!B) return fail(MECH_E_INVALID, "batch is NULL");
    return step_impl(B, n_steps);
}

int batch_poll(MechBatch* B, int32_t* done_slots, int32_t capacity, int32_t* n_done)
{
    if (!B || !n_done) return fail(MECH_E_INVALID, "batch or n_done is NULL");
    int32_t k = 0;
    for (int32_t id : B->order) {
        HostSlot& s = B->slots[id];
        if (s.retired || s.reported || !s.done_recorded) continue;
        hipError_t q = hipEventQuery(s.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return fail(MECH_E_DEVICE, "hipEventQuery failed: %s", hipGetErrorString(q));
        if (k < capacity && done_slots) done_slots[k] = id;
        ++k;
        s.reported = true;
    }
    *n_done = k;
    return MECH_OK;
}

int batch_read(MechBatch* B, int32_t slot, double* pos, double* vel, int64_t n_cells)
{
    if (!B) return fail(MECH_E_INVALID, "batch is NULL");
    return read_slot(B, slot, pos, vel, n_cells);
}

int batch_retire(MechBatch* B, int32_t slot)
{
    if (!B) return fail(MECH_E_INVALID, "batch is NULL");
    if (slot < 0 || slot >= B->cap_slots || !B->slots[slot].used || B->slots[slot].retired)
        return fail(MECH_E_INVALID, "slot %d holds no simulation", slot);
    HIP_TRY(hipSetDevice(B->device));
    HostSlot& s = B->slots[slot];
    s.retired = true;
    s.d.steps_left = 0;  // frozen until the next repack drops it
    push_slot(B, slot);
    HIP_TRY(hipGetLastError());
    return MECH_OK;
}

int batch_slot_info(MechBatch* B, int32_t slot, int64_t* n_cells, int64_t* steps_left)
{
    if (!B) return fail(MECH_E_INVALID, "batch is NULL");
    if (slot < 0 || slot >= B->cap_slots || !B->slots[slot].used || B->slots[slot].retired)
        return fail(MECH_E_INVALID, "slot %d holds no simulation", slot);
    if (n_cells) *n_cells = B->slots[slot].d.n_cells;
    if (steps_left) *steps_left = B->slots[slot].d.steps_left;
    return MECH_OK;
}

int batch_info(MechBatch* B, int64_t* n_cells, int64_t* n_voxels, int32_t* n_live, int64_t* free_cells,
               int64_t* free_voxels)
{
    if (!B) return fail(MECH_E_INVALID, "batch is NULL");
    int64_t lc = 0, lv = 0;
    int32_t nl = 0;
    for (int32_t id : B->order)
        if (!B->slots[id].retired) {
            const SlotDesc& d = B->slots[id].d;
            lc += d.n_cells;
            lv += (int64_t)d.nx * d.ny * d.nz;
            ++nl;
        }
    if (n_cells) *n_cells = B->n_cells;
    if (n_voxels) *n_voxels = B->n_voxels;
    if (n_live) *n_live = nl;
    if (free_cells) *free_cells = B->cap_cells - lc;
    if (free_voxels) *free_voxels = B->cap_voxels - lv;
    return MECH_OK;
}

int batch_stats(MechBatch* B, int64_t* steps, int64_t* interactions, int64_t* candidates)
{
    if (!B) return fail(MECH_E_INVALID, "batch is NULL");
    return stats_impl(B, steps, interactions, candidates);
}

int batch_profile(MechBatch* B, int64_t n_steps, double* phase_ms)
{
    if (!B) return fail(MECH_E_INVALID, "batch is NULL");
    return profile_impl(B, n_steps, phase_ms);
}

int batch_set_flags(MechBatch* B, int32_t flags)
{
    if (!B) return fail(MECH_E_INVALID, "batch is NULL");
    MechParams p = B->prm;
    p.flags = flags;
    int rc = validate_physics(&p);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(B->device));
    HIP_TRY(hipStreamSynchronize(B->stream));
    drop_graphs(B);
    B->prm.flags = flags;
    return MECH_OK;
}

int batch_get_tuning(MechBatch* B, MechTuning* out)
{
    if (!B || !out) return fail(MECH_E_INVALID, "batch or out is NULL");
    *out = B->tune;
    out->force_kernel = B->prm.flags & MECH_FORCE_KERNEL_MASK;
    return MECH_OK;
}

int batch_set_tuning(MechBatch* B, const MechTuning* t)
{
    if (!B || !t) return fail(MECH_E_INVALID, "batch or tuning is NULL");
    if (t->force_kernel != 0 && t->force_kernel != MECH_FLAG_SIMPLE_FORCE && t->force_kernel != MECH_FLAG_VOXEL_FORCE &&
        t->force_kernel != MECH_FLAG_PRUNED_FORCE)
        return fail(MECH_E_INVALID, "force_kernel %d unknown", t->force_kernel);
    if (t->block_waves != 1 && t->block_waves != 2 && t->block_waves != 4 && t->block_waves != 8)
        return fail(MECH_E_INVALID, "block_waves %d not in {1, 2, 4, 8}", t->block_waves);
    if (t->unroll != 2 && t->unroll != 4 && t->unroll != 8)
        return fail(MECH_E_INVALID, "unroll %d not in {2, 4, 8}", t->unroll);
    if (t->blocks_per_cu < 0 || t->blocks_per_cu > 64)
        return fail(MECH_E_INVALID, "blocks_per_cu %d not in [0, 64]", t->blocks_per_cu);
    if (t->list_len != 0 && t->list_len != 16 && t->list_len != 32 && t->list_len != 64)
        return fail(MECH_E_INVALID, "list_len %d not in {0, 16, 32, 64}", t->list_len);
    if (t->block_waves == 8 && t->list_len == 64)
        return fail(MECH_E_INVALID, "8 waves per workgroup with 64-entry lists exceed a compute unit's LDS");
    HIP_TRY(hipSetDevice(B->device));
    HIP_TRY(hipStreamSynchronize(B->stream));
    drop_graphs(B);
    B->tune = *t;
    B->prm.flags = (B->prm.flags & ~MECH_FORCE_KERNEL_MASK) | t->force_kernel;
    return MECH_OK;
}

int batch_sync(MechBatch* B)
{
    if (!B) return fail(MECH_E_INVALID, "batch is NULL");
    HIP_TRY(hipSetDevice(B->device));
    return sync_check(B);
}

void* batch_stream(MechBatch* B) { return B ? (void*)B->stream : nullptr; }

int destroy_batch(MechBatch* B)
{
    if (!B) return MECH_OK;
    (void)hipSetDevice(B->device);
    hipError_t e = B->stream ? hipStreamSynchronize(B->stream) : hipSuccess;
    release(B);
    if (e != hipSuccess) return fail(MECH_E_DEVICE, "stream error at destroy: %s", hipGetErrorString(e));
    return MECH_OK;
}

}  // extern "C"
