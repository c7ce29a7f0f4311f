// microenv.hip -- gfx950 kernels and C-ABI runtime of the microenvironment solver
// (libmech.so, declared in include/microenv.h).
//
// One solver step, on the handle's stream:
//   k_solve_x      implicit solve along x of every mesh line (lines are contiguous rows
//                  of nx values: a block stages 64 of them into LDS with coalesced
//                  loads, each lane runs the Thomas recurrences on its row there, and
//                  the block writes them back coalesced)
//   k_solve_yz     implicit solve along y or z: lanes take lines whose voxels are
//                  adjacent in x (consecutive addresses), so every load and store is
//                  coalesced across the wave; each lane loads its line into its own LDS
//                  column (lane-interleaved, no bank conflicts), runs the recurrences
//                  there and stores the line back
// Lines longer than 128 voxels are solved in place in device memory instead.
// and on request
//   k_gradients    central differences (one-sided on the faces) of every substrate along
//                  every axis
// The paper finds the CPU loops of the solver and of the gradients imbalanced because
// only the 75 z planes were shared among the threads, and fixes it by sharing the 75 x 75
// (z, y) lines instead (Section 5.2).  Here every line of the mesh is its own lane: 5625
// lines per substrate and axis on a 75^3 mesh.
//
// The tridiagonal matrices are the same for every line of one substrate and axis, so
// their elimination factors are computed once on the host (in FP64, when the handle is
// made) and the kernels only run the two recurrences of the Thomas algorithm:
//   y_0 = rho_0 / m_0,  y_i = (rho_i + r y_{i-1}) / m_i,  u_{n-1} = y_{n-1},
//   u_i = y_i - c_i u_{i+1},
// with m_i the eliminated diagonal and c_i = -r / m_i (c_{n-1} = 0), stored as c_i and
// 1 / m_i.  This differs from the textbook's division at each step only by rounding.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "microenv.h"

int mech_report_error(int code, const char* text);   // mech.hip: sets mech_last_error()

namespace {

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return mech_report_error(code, buf);
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(MECH_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

constexpr int LINES = 64;          // mesh lines per block (one wave64)
constexpr int LDS_MAX_N = 128;     // longest line staged in LDS (64 x 128 doubles = 64 KiB)
constexpr int SEG_MAX = 8;         // segments per line in k_solve_seg
constexpr int SEG_MIN_LEN = 10;    // shortest segment worth a thread of its own
constexpr int SEG_MAX_N = 112;     // longest line of k_solve_seg: the tile and the maps in LDS
constexpr int SEG_LEN_MAX = 16;    // longest segment: ceil(112 / 8) = 14 fits
constexpr int GRAD_BLOCK = 256;
constexpr int MAX_DIM = 4096;
constexpr unsigned N_XCD = 8;      // MI355X: 8 accelerator complex dies, each with its own L2

// Workgroups reach the XCDs round robin; renumber them so that each XCD takes one
// contiguous run of the nb tiles, and tiles that share cache lines share an L2.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nb)
{
    const unsigned xcd = b % N_XCD, k = b / N_XCD, q = nb / N_XCD, r = nb % N_XCD;
    return xcd < r ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

// Elimination factors of one substrate and axis: c[n] then inv_m[n], and r.
struct Factors {
    const double* c;
    const double* inv_m;
    double r;
};

struct SolveArgs {
    double* rho;
    const double* fac;       // [s][axis][2][nmax]: c, then 1/m
    const double* r;         // [s][axis]
    int nmax;
    int nx, ny, nz;
    int64_t V;
};

__device__ __forceinline__ Factors factors(const SolveArgs& a, int s, int axis)
{
    const double* f = a.fac + ((size_t)(s * 3 + axis) * 2) * (size_t)a.nmax;
    return Factors{f, f + a.nmax, a.r[s * 3 + axis]};
}

// The two recurrences on one line of n values: read(i) gives the right-hand side, the
// forward values go to tmp(i) and the solution to out(i) (all three may be the same
// array: every index is read before it is written).  The operands are fetched CH at a
// time ahead of the dependent arithmetic, so their latency is paid once per chunk.  The
// first forward value comes out of the general formula with y = 0: fl(rho_0 + r 0) is
// rho_0.
constexpr int CH = 8;

template <typename Rd, typename Tw, typename Tr, typename Ow>
__device__ __forceinline__ void thomas(int n, const Factors& F, Rd read, Tw tmp_w, Tr tmp_r, Ow out)
{
    double y = 0.0;
    for (int i0 = 0; i0 < n; i0 += CH) {
        double v[CH], m[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k)
            if (i0 + k < n) {
                v[k] = read(i0 + k);
                m[k] = F.inv_m[i0 + k];
            }
#pragma unroll
        for (int k = 0; k < CH; ++k)
            if (i0 + k < n) {
                y = (v[k] + F.r * y) * m[k];
                tmp_w(i0 + k, y);
            }
    }
    double u = y;
    out(n - 1, u);
    for (int i1 = n - 1; i1 > 0; i1 -= CH) {   // indices i1 - 1 down to i1 - CH
        double t[CH], c[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k)
            if (i1 - 1 - k >= 0) {
                t[k] = tmp_r(i1 - 1 - k);
                c[k] = F.c[i1 - 1 - k];
            }
#pragma unroll
        for (int k = 0; k < CH; ++k)
            if (i1 - 1 - k >= 0) {
                u = t[k] - c[k] * u;
                out(i1 - 1 - k, u);
            }
    }
}

// Solve along x.  Line L (over all substrates) is the contiguous row rho[L nx ...]; a
// block takes 64 consecutive lines, so its rows are one contiguous range of memory,
// loaded into LDS and stored back with consecutive lanes on consecutive addresses.
template <bool LDS>
__global__ __launch_bounds__(LINES) void k_solve_x(SolveArgs a, int64_t lines)
{
    extern __shared__ double sh[];
    const int nx = a.nx;
    const int64_t L0 = (int64_t)blockIdx.x * LINES;
    const int cnt = (int)min<int64_t>(LINES, lines - L0);
    double* g = a.rho + L0 * nx;
    const int lane = threadIdx.x;
    const int64_t lines_per_sub = (int64_t)a.ny * a.nz;
    if constexpr (LDS) {
        const int tot = cnt * nx;
#pragma unroll 8
        for (int t = lane; t < tot; t += LINES) sh[t] = g[t];
        __syncthreads();
        if (lane < cnt) {
            const Factors F = factors(a, (int)((L0 + lane) / lines_per_sub), 0);
            double* u = sh + lane * nx;
            auto rd = [&](int i) { return u[i]; };
            auto wr = [&](int i, double v) { u[i] = v; };
            thomas(nx, F, rd, wr, rd, wr);
        }
        __syncthreads();
#pragma unroll 8
        for (int t = lane; t < tot; t += LINES) g[t] = sh[t];
    } else {
        // rows longer than LDS holds: each lane walks its row in place
        if (lane < cnt) {
            const Factors F = factors(a, (int)((L0 + lane) / lines_per_sub), 0);
            double* u = g + (int64_t)lane * nx;
            auto rd = [&](int i) { return u[i]; };
            auto wr = [&](int i, double v) { u[i] = v; };
            thomas(nx, F, rd, wr, rd, wr);
        }
    }
}

// Solve along y (AXIS 1) or z (AXIS 2).  Lines of one substrate are numbered with x
// fastest: along z, line l starts at voxel l of the first z plane; along y, line
// l = i + nx k starts at (i, 0, k).  Consecutive lanes read consecutive addresses.  With
// LDS the lane's line is first loaded into its LDS column (lane-interleaved: no bank
// conflicts), every load in flight at once, solved there and stored back.
template <int AXIS, bool LDS>
__global__ __launch_bounds__(LINES) void k_solve_yz(SolveArgs a, int64_t lines)
{
    extern __shared__ double sh[];
    const int64_t L = (int64_t)blockIdx.x * LINES + threadIdx.x;
    if (L >= lines) return;
    const int64_t lines_per_sub = AXIS == 1 ? (int64_t)a.nx * a.nz : (int64_t)a.nx * a.ny;
    const int s = (int)(L / lines_per_sub);
    const int64_t l = L - (int64_t)s * lines_per_sub;
    int64_t base;
    int64_t stride;
    int n;
    if (AXIS == 1) {
        const int64_t i = l % a.nx, k = l / a.nx;
        base = (int64_t)s * a.V + k * a.nx * a.ny + i;
        stride = a.nx;
        n = a.ny;
    } else {
        base = (int64_t)s * a.V + l;
        stride = (int64_t)a.nx * a.ny;
        n = a.nz;
    }
    double* p = a.rho + base;
    const Factors F = factors(a, s, AXIS);
    if constexpr (LDS) {
        double* w = sh + threadIdx.x;
#pragma unroll 16
        for (int i = 0; i < n; ++i) w[i * LINES] = p[i * stride];
        auto rd = [&](int i) { return w[i * LINES]; };
        auto wr = [&](int i, double v) { w[i * LINES] = v; };
        thomas(n, F, rd, wr, rd, wr);
#pragma unroll 16
        for (int i = 0; i < n; ++i) p[i * stride] = w[i * LINES];
    } else {
        auto rd = [&](int i) { return p[i * stride]; };
        auto wr = [&](int i, double v) { p[i * stride] = v; };
        thomas(n, F, rd, wr, rd, wr);
    }
}

// Solve along any axis with every line cut into segments (n <= SEG_MAX_N).  A block takes
// LB lines and nseg segments of each: thread t works on line t % LB and segment t / LB,
// so a line's segments run in parallel.  Both recurrences are affine in their running
// value (y_i = m_i r y_{i-1} + m_i rho_i forward, u_i = y_i - c_i u_{i+1} back), so each
// thread first composes its segment's map, the maps of the segments before it give the
// value its segment starts from (at most nseg - 1 compositions), and the segment is then
// recomputed from that value with the recurrence as written.  The chain of dependent
// operations per line shrinks from 2n to about 4n / nseg + 2 nseg.  A thread holds its
// segment's values and factors in registers from one batch of loads.  The block's lines
// sit in LDS as tile[i][l]; loads and stores run with consecutive threads on consecutive
// addresses (whole contiguous rows along x; along y and z the LB lines of one index i).
template <int AXIS, int LB>
__global__ __launch_bounds__(SEG_MAX * LINES) void k_solve_seg(SolveArgs a, int64_t lines, int seg_len)
{
    extern __shared__ double sh[];
    const int n = AXIS == 0 ? a.nx : AXIS == 1 ? a.ny : a.nz;
    const int nseg = blockDim.x / LB;
    constexpr int LS = LB + 1;               // row stride: odd, so a column walk spreads over banks
    double* tile = sh;                       // [n][LS]
    double* mp = sh + (size_t)n * LS;        // [nseg][LB] composed maps: y_out = P y_in + Q
    double* mq = mp + (size_t)nseg * LB;
    const int l = threadIdx.x % LB, w = threadIdx.x / LB;
    const int64_t L0 = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * LB;
    const int cnt = (int)min<int64_t>(LB, lines - L0);
    const int64_t lines_per_sub = AXIS == 0 ? (int64_t)a.ny * a.nz
                                            : AXIS == 1 ? (int64_t)a.nx * a.nz : (int64_t)a.nx * a.ny;
    // first element and stride of line L0 + l (valid for l < cnt)
    int64_t base = 0, stride = 1;
    int s = 0;
    {
        const int64_t L = L0 + min(l, cnt - 1);
        s = (int)(L / lines_per_sub);
        const int64_t q = L - (int64_t)s * lines_per_sub;
        if (AXIS == 0) {
            base = L * a.nx;
        } else if (AXIS == 1) {
            base = (int64_t)s * a.V + (q / a.nx) * a.nx * a.ny + q % a.nx;
            stride = a.nx;
        } else {
            base = (int64_t)s * a.V + q;
            stride = (int64_t)a.nx * a.ny;
        }
    }
    if (AXIS == 0) {
        const double* g = a.rho + L0 * a.nx;
        const int tot = cnt * n;
        for (int t = threadIdx.x; t < tot; t += blockDim.x) tile[(t % n) * LS + t / n] = g[t];
    } else if (l < cnt) {
        const double* p = a.rho + base;
#pragma unroll 4
        for (int i = w; i < n; i += nseg) tile[i * LS + l] = p[i * stride];
    }
    __syncthreads();
    const Factors F = factors(a, s, AXIS);
    const int i0 = min(n, w * seg_len), len = min(n, i0 + seg_len) - i0;
    const bool on = l < cnt;
    // the segment's values and factors, all loads issued before the arithmetic
    double v[SEG_LEN_MAX], m[SEG_LEN_MAX], c[SEG_LEN_MAX];
#pragma unroll
    for (int k = 0; k < SEG_LEN_MAX; ++k)
        if (k < len) {
            v[k] = tile[(i0 + k) * LS + l];
            m[k] = F.inv_m[i0 + k];
            c[k] = F.c[i0 + k];
        }
    // forward: the segment's map y_out = P y_in + Q, the starting value, the recurrence
    double P = 1.0, Q = 0.0;
#pragma unroll
    for (int k = 0; k < SEG_LEN_MAX; ++k)
        if (k < len) {
            P = m[k] * F.r * P;
            Q = (v[k] + F.r * Q) * m[k];
        }
    mp[w * LB + l] = P;
    mq[w * LB + l] = Q;
    __syncthreads();
    double y = 0.0;
    if (on)
        for (int j = 0; j < w; ++j) y = mp[j * LB + l] * y + mq[j * LB + l];
#pragma unroll
    for (int k = 0; k < SEG_LEN_MAX; ++k)
        if (k < len) {
            y = (v[k] + F.r * y) * m[k];
            v[k] = y;
        }
    __syncthreads();   // every thread has read the forward maps
    // back substitution: the map from the value after the segment down to its first
    P = 1.0;
    Q = 0.0;
#pragma unroll
    for (int k = SEG_LEN_MAX - 1; k >= 0; --k)
        if (k < len) {
            P = -c[k] * P;
            Q = v[k] - c[k] * Q;
        }
    mp[w * LB + l] = P;
    mq[w * LB + l] = Q;
    __syncthreads();
    double u = 0.0;
    if (on)
        for (int j = nseg - 1; j > w; --j) u = mp[j * LB + l] * u + mq[j * LB + l];
#pragma unroll
    for (int k = SEG_LEN_MAX - 1; k >= 0; --k)
        if (k < len) {
            u = v[k] - c[k] * u;
            tile[(i0 + k) * LS + l] = u;
        }
    __syncthreads();
    if (AXIS == 0) {
        double* g = a.rho + L0 * a.nx;
        const int tot = cnt * n;
        for (int t = threadIdx.x; t < tot; t += blockDim.x) g[t] = tile[(t % n) * LS + t / n];
    } else if (l < cnt) {
        double* p = a.rho + base;
#pragma unroll 4
        for (int i = w; i < n; i += nseg) p[i * stride] = tile[i * LS + l];
    }
}

// Gradients: one thread per voxel and substrate (grid-stride), x fastest.
__global__ __launch_bounds__(GRAD_BLOCK) void k_gradients(const double* __restrict__ rho, double* __restrict__ grad,
                                                          int nx, int ny, int nz, int64_t V, int64_t total,
                                                          double inv_dx, double inv_2dx)
{
    for (int64_t t = (int64_t)blockIdx.x * GRAD_BLOCK + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * GRAD_BLOCK) {
        const int64_t s = t / V, v = t - s * V;
        const int i = (int)(v % nx);
        const int j = (int)((v / nx) % ny);
        const int k = (int)(v / ((int64_t)nx * ny));
        const double* u = rho + s * V + v;
        const int c[3] = {i, j, k};
        const int n[3] = {nx, ny, nz};
        const int64_t st[3] = {1, nx, (int64_t)nx * ny};
        double* g = grad + s * 3 * V + v;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            double val;
            if (n[ax] == 1) val = 0.0;
            else if (c[ax] == 0) val = (u[st[ax]] - u[0]) * inv_dx;
            else if (c[ax] == n[ax] - 1) val = (u[0] - u[-st[ax]]) * inv_dx;
            else val = (u[st[ax]] - u[-st[ax]]) * inv_2dx;
            g[ax * V] = val;
        }
    }
}

}  // namespace

struct MechMicroenv {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    MechMicroenvParams p{};
    int64_t V = 0;
    int nmax = 0;
    double* rho = nullptr;
    double* grad = nullptr;
    double* fac = nullptr;
    double* rr = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev[5] = {};
    int grad_blocks = 0;
    int cus = 256;
};

namespace {

int validate(const MechMicroenvParams* p, int64_t* V)
{
    if (!p) return fail(MECH_E_INVALID, "params is NULL");
    if (p->abi_version != MECH_ABI_VERSION)
        return fail(MECH_E_INVALID, "abi_version %d, library %d", p->abi_version, MECH_ABI_VERSION);
    if (p->reserved != 0) return fail(MECH_E_INVALID, "reserved must be 0");
    if (p->n_substrates < 1 || p->n_substrates > MECH_MAX_SUBSTRATES)
        return fail(MECH_E_INVALID, "n_substrates %d outside 1..%d", p->n_substrates, MECH_MAX_SUBSTRATES);
    int64_t v = 1;
    for (int a = 0; a < 3; ++a) {
        if (p->dims[a] < 1 || p->dims[a] > MAX_DIM)
            return fail(MECH_E_INVALID, "dims[%d] = %d outside 1..%d", a, p->dims[a], MAX_DIM);
        v *= p->dims[a];
    }
    if (v >= (int64_t(1) << 31)) return fail(MECH_E_INVALID, "%lld voxels: at most 2^31 - 1", (long long)v);
    if (!(std::isfinite(p->voxel_size) && p->voxel_size > 0.0)) return fail(MECH_E_INVALID, "voxel_size must be > 0");
    if (!(std::isfinite(p->dt) && p->dt >= 0.0)) return fail(MECH_E_INVALID, "dt must be finite and >= 0");
    for (int s = 0; s < p->n_substrates; ++s) {
        if (!(std::isfinite(p->diffusion[s]) && p->diffusion[s] >= 0.0))
            return fail(MECH_E_INVALID, "diffusion[%d] must be finite and >= 0", s);
        if (!(std::isfinite(p->decay[s]) && p->decay[s] >= 0.0))
            return fail(MECH_E_INVALID, "decay[%d] must be finite and >= 0", s);
    }
    *V = v;
    return MECH_OK;
}

// Elimination factors of the system of one substrate and axis (see the file header).
void eliminate(int n, double r, double b, double* c, double* inv_m)
{
    if (n == 1) {
        c[0] = 0.0;
        inv_m[0] = 1.0 / b;
        return;
    }
    double m = b + r;
    c[0] = -r / m;
    inv_m[0] = 1.0 / m;
    for (int i = 1; i < n; ++i) {
        const double diag = (i == n - 1) ? b + r : b + 2.0 * r;
        m = diag + r * c[i - 1];
        c[i] = (i == n - 1) ? 0.0 : -r / m;
        inv_m[i] = 1.0 / m;
    }
}

void release(MechMicroenv* E)
{
    if (E->exec) (void)hipGraphExecDestroy(E->exec);
    if (E->graph) (void)hipGraphDestroy(E->graph);
    for (auto& e : E->ev)
        if (e) (void)hipEventDestroy(e);
    if (E->rho) (void)hipFree(E->rho);
    if (E->grad) (void)hipFree(E->grad);
    if (E->fac) (void)hipFree(E->fac);
    if (E->rr) (void)hipFree(E->rr);
    if (E->own_stream && E->stream) (void)hipStreamDestroy(E->stream);
    delete E;
}

SolveArgs solve_args(const MechMicroenv* E)
{
    return SolveArgs{E->rho, E->fac, E->rr, E->nmax, E->p.dims[0], E->p.dims[1], E->p.dims[2], E->V};
}

template <int AXIS, int LB>
void launch_seg(MechMicroenv* E, const SolveArgs& a, int64_t lines, int n)
{
    const int nseg = std::min(SEG_MAX, std::max(1, (n + SEG_MIN_LEN - 1) / SEG_MIN_LEN));
    const int seg_len = (n + nseg - 1) / nseg;
    const unsigned blocks = (unsigned)((lines + LB - 1) / LB);
    const size_t shm = ((size_t)n * (LB + 1) + 2 * (size_t)nseg * LB) * sizeof(double);
    k_solve_seg<AXIS, LB><<<blocks, nseg * LB, shm, E->stream>>>(a, lines, seg_len);
}

template <int AXIS>
void launch_seg_lb(MechMicroenv* E, const SolveArgs& a, int64_t lines, int n)
{
    // lines per block: as many as still give every compute unit two blocks
    if (lines >= (int64_t)32 * 2 * E->cus)
        launch_seg<AXIS, 32>(E, a, lines, n);
    else
        launch_seg<AXIS, 16>(E, a, lines, n);
}

// One launch of the solve along `axis`.
int launch_solve(MechMicroenv* E, int axis)
{
    const SolveArgs a = solve_args(E);
    const int64_t ns = E->p.n_substrates;
    const int n = E->p.dims[axis];
    const int64_t lines = ns * (E->V / n);
    // Segments pay when the lines alone would leave compute units idle (fewer lines than
    // one wave per compute unit holds lanes); with more lines the chip is full anyway and
    // the per-line walk does half the arithmetic.
    const int nseg = std::min(SEG_MAX, std::max(1, (n + SEG_MIN_LEN - 1) / SEG_MIN_LEN));
    if (n <= SEG_MAX_N && (n + nseg - 1) / nseg <= SEG_LEN_MAX && lines <= (int64_t)LINES * E->cus) {
        if (axis == 0) launch_seg_lb<0>(E, a, lines, n);
        else if (axis == 1) launch_seg_lb<1>(E, a, lines, n);
        else launch_seg_lb<2>(E, a, lines, n);
        HIP_TRY(hipGetLastError());
        return MECH_OK;
    }
    const bool lds = n <= LDS_MAX_N;
    const unsigned blocks = (unsigned)((lines + LINES - 1) / LINES);
    const size_t shm = lds ? (size_t)LINES * (size_t)n * sizeof(double) : 0;
    if (axis == 0) {
        if (lds) k_solve_x<true><<<blocks, LINES, shm, E->stream>>>(a, lines);
        else k_solve_x<false><<<blocks, LINES, 0, E->stream>>>(a, lines);
    } else if (axis == 1) {
        if (lds) k_solve_yz<1, true><<<blocks, LINES, shm, E->stream>>>(a, lines);
        else k_solve_yz<1, false><<<blocks, LINES, 0, E->stream>>>(a, lines);
    } else {
        if (lds) k_solve_yz<2, true><<<blocks, LINES, shm, E->stream>>>(a, lines);
        else k_solve_yz<2, false><<<blocks, LINES, 0, E->stream>>>(a, lines);
    }
    HIP_TRY(hipGetLastError());
    return MECH_OK;
}

int launch_step(MechMicroenv* E)
{
    for (int axis = 0; axis < 3; ++axis) {
        int rc = launch_solve(E, axis);
        if (rc) return rc;
    }
    return MECH_OK;
}

int launch_gradients(MechMicroenv* E)
{
    const double dx = E->p.voxel_size;
    k_gradients<<<E->grad_blocks, GRAD_BLOCK, 0, E->stream>>>(E->rho, E->grad, E->p.dims[0], E->p.dims[1],
                                                              E->p.dims[2], E->V, E->V * E->p.n_substrates,
                                                              1.0 / dx, 1.0 / (2.0 * dx));
    HIP_TRY(hipGetLastError());
    return MECH_OK;
}

int build_graph(MechMicroenv* E)
{
    HIP_TRY(hipStreamBeginCapture(E->stream, hipStreamCaptureModeThreadLocal));
    int rc = launch_step(E);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(E->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(MECH_E_DEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    E->graph = g;
    HIP_TRY(hipGraphInstantiate(&E->exec, g, nullptr, nullptr, 0));
    return MECH_OK;
}

int check_values(const double* v, int64_t n, const char* what)
{
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(v[k])) return fail(MECH_E_NONFINITE, "%s[%lld] is not finite", what, (long long)k);
    return MECH_OK;
}

}  // namespace

extern "C" {

int create_microenvironment(const MechMicroenvParams* params, const double* density, void* hip_stream,
                            MechMicroenv** out)
{
    if (!out) return fail(MECH_E_INVALID, "out is NULL");
    *out = nullptr;
    int64_t V = 0;
    int rc = validate(params, &V);
    if (rc) return rc;
    const int64_t nv = V * params->n_substrates;
    if (density) {
        for (int64_t k = 0; k < nv; ++k)
            if (!std::isfinite(density[k]))
                return fail(MECH_E_INVALID, "density[%lld] is not finite", (long long)k);
    }
    MechMicroenv* E = new (std::nothrow) MechMicroenv();
    if (!E) return fail(MECH_E_NOMEM, "out of host memory");
    auto bail = [&](int code) {
        release(E);
        return code;
    };
    E->p = *params;
    E->V = V;
    E->nmax = std::max(params->dims[0], std::max(params->dims[1], params->dims[2]));
    if (hipGetDevice(&E->device) != hipSuccess) return bail(fail(MECH_E_DEVICE, "no HIP device"));
    if (hip_stream) {
        E->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&E->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(MECH_E_DEVICE, "hipStreamCreate failed"));
        E->own_stream = true;
    }
    for (auto& e : E->ev)
        if (hipEventCreate(&e) != hipSuccess) return bail(fail(MECH_E_DEVICE, "hipEventCreate failed"));
    const size_t nfac = (size_t)params->n_substrates * 3 * 2 * (size_t)E->nmax;
    if (hipMalloc(&E->rho, (size_t)nv * sizeof(double)) != hipSuccess ||
        hipMalloc(&E->grad, (size_t)nv * 3 * sizeof(double)) != hipSuccess ||
        hipMalloc(&E->fac, nfac * sizeof(double)) != hipSuccess ||
        hipMalloc(&E->rr, (size_t)params->n_substrates * 3 * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(MECH_E_NOMEM, "device allocation of %lld values failed", (long long)(4 * nv)));
    }
    // elimination factors, per substrate and axis
    std::vector<double> fac(nfac, 0.0), rr((size_t)params->n_substrates * 3);
    const double dx = params->voxel_size;
    for (int s = 0; s < params->n_substrates; ++s) {
        const double r = params->diffusion[s] * params->dt / (dx * dx);
        const double b = 1.0 + params->decay[s] * params->dt / 3.0;
        for (int a = 0; a < 3; ++a) {
            double* f = fac.data() + ((size_t)(s * 3 + a) * 2) * (size_t)E->nmax;
            eliminate(params->dims[a], r, b, f, f + E->nmax);
            rr[(size_t)s * 3 + a] = r;
        }
    }
    if (hipMemcpyAsync(E->fac, fac.data(), nfac * sizeof(double), hipMemcpyHostToDevice, E->stream) != hipSuccess ||
        hipMemcpyAsync(E->rr, rr.data(), rr.size() * sizeof(double), hipMemcpyHostToDevice, E->stream) != hipSuccess)
        return bail(fail(MECH_E_DEVICE, "copy of the factors failed"));
    if (density) {
        if (hipMemcpyAsync(E->rho, density, (size_t)nv * sizeof(double), hipMemcpyHostToDevice, E->stream) != hipSuccess)
            return bail(fail(MECH_E_DEVICE, "copy of the densities failed"));
    } else if (hipMemsetAsync(E->rho, 0, (size_t)nv * sizeof(double), E->stream) != hipSuccess) {
        return bail(fail(MECH_E_DEVICE, "hipMemsetAsync failed"));
    }
    if (hipMemsetAsync(E->grad, 0, (size_t)nv * 3 * sizeof(double), E->stream) != hipSuccess ||
        hipStreamSynchronize(E->stream) != hipSuccess)
        return bail(fail(MECH_E_DEVICE, "initialisation failed"));
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, E->device) != hipSuccess || cus < 1)
        cus = 256;
    E->cus = cus;
    const int64_t need = (nv + GRAD_BLOCK - 1) / GRAD_BLOCK;
    E->grad_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)cus * 16));
    *out = E;
    return MECH_OK;
}

int microenvironment_step(MechMicroenv* E, int64_t n_steps)
{
    if (!E) return fail(MECH_E_INVALID, "handle is NULL");
    if (n_steps < 0) return fail(MECH_E_INVALID, "n_steps < 0");
    if (n_steps == 0) return MECH_OK;
    HIP_TRY(hipSetDevice(E->device));
    if (!E->exec) {
        int rc = build_graph(E);
        if (rc) return rc;
    }
    for (int64_t t = 0; t < n_steps; ++t) HIP_TRY(hipGraphLaunch(E->exec, E->stream));
    return MECH_OK;
}

int microenvironment_gradients(MechMicroenv* E)
{
    if (!E) return fail(MECH_E_INVALID, "handle is NULL");
    HIP_TRY(hipSetDevice(E->device));
    return launch_gradients(E);
}

int read_density(MechMicroenv* E, double* density, int64_t n_values)
{
    if (!E || !density) return fail(MECH_E_INVALID, "handle or array is NULL");
    const int64_t nv = E->V * E->p.n_substrates;
    if (n_values != nv) return fail(MECH_E_INVALID, "n_values %lld, the mesh holds %lld", (long long)n_values, (long long)nv);
    HIP_TRY(hipSetDevice(E->device));
    HIP_TRY(hipMemcpyAsync(density, E->rho, (size_t)nv * sizeof(double), hipMemcpyDeviceToHost, E->stream));
    HIP_TRY(hipStreamSynchronize(E->stream));
    return check_values(density, nv, "density");
}

int read_gradients(MechMicroenv* E, double* grad, int64_t n_values)
{
    if (!E || !grad) return fail(MECH_E_INVALID, "handle or array is NULL");
    const int64_t nv = 3 * E->V * E->p.n_substrates;
    if (n_values != nv) return fail(MECH_E_INVALID, "n_values %lld, the gradients hold %lld", (long long)n_values, (long long)nv);
    HIP_TRY(hipSetDevice(E->device));
    HIP_TRY(hipMemcpyAsync(grad, E->grad, (size_t)nv * sizeof(double), hipMemcpyDeviceToHost, E->stream));
    HIP_TRY(hipStreamSynchronize(E->stream));
    return check_values(grad, nv, "grad");
}

int write_density(MechMicroenv* E, const double* density, int64_t n_values)
{
    if (!E || !density) return fail(MECH_E_INVALID, "handle or array is NULL");
    const int64_t nv = E->V * E->p.n_substrates;
    if (n_values != nv) return fail(MECH_E_INVALID, "n_values %lld, the mesh holds %lld", (long long)n_values, (long long)nv);
    for (int64_t k = 0; k < nv; ++k)
        if (!std::isfinite(density[k])) return fail(MECH_E_INVALID, "density[%lld] is not finite", (long long)k);
    HIP_TRY(hipSetDevice(E->device));
    HIP_TRY(hipStreamSynchronize(E->stream));
    HIP_TRY(hipMemcpyAsync(E->rho, density, (size_t)nv * sizeof(double), hipMemcpyHostToDevice, E->stream));
    HIP_TRY(hipStreamSynchronize(E->stream));
    return MECH_OK;
}

int microenvironment_profile(MechMicroenv* E, int64_t n_steps, double ms[4])
{
    if (!E || !ms) return fail(MECH_E_INVALID, "handle or ms is NULL");
    if (n_steps < 1) return fail(MECH_E_INVALID, "n_steps < 1");
    HIP_TRY(hipSetDevice(E->device));
    double tot[4] = {0, 0, 0, 0};
    for (int64_t t = 0; t < n_steps; ++t) {
        HIP_TRY(hipEventRecord(E->ev[0], E->stream));
        for (int axis = 0; axis < 3; ++axis) {
            int rc = launch_solve(E, axis);
            if (rc) return rc;
            HIP_TRY(hipEventRecord(E->ev[axis + 1], E->stream));
        }
        HIP_TRY(hipEventSynchronize(E->ev[3]));
        for (int axis = 0; axis < 3; ++axis) {
            float f = 0.0f;
            HIP_TRY(hipEventElapsedTime(&f, E->ev[axis], E->ev[axis + 1]));
            tot[axis] += f;
        }
    }
    HIP_TRY(hipEventRecord(E->ev[0], E->stream));
    int rc = launch_gradients(E);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(E->ev[4], E->stream));
    HIP_TRY(hipEventSynchronize(E->ev[4]));
    float f = 0.0f;
    HIP_TRY(hipEventElapsedTime(&f, E->ev[0], E->ev[4]));
    for (int k = 0; k < 3; ++k) ms[k] = tot[k] / (double)n_steps;
    ms[3] = f;
    return MECH_OK;
}

int microenvironment_device_arrays(MechMicroenv* E, double** density, double** grad)
{
    if (!E) return fail(MECH_E_INVALID, "handle is NULL");
    if (density) *density = E->rho;
    if (grad) *grad = E->grad;
    return MECH_OK;
}

void* microenvironment_stream(MechMicroenv* E) { return E ? (void*)E->stream : nullptr; }

int destroy_microenvironment(MechMicroenv* E)
{
    if (!E) return MECH_OK;
    (void)hipSetDevice(E->device);
    const hipError_t e = E->stream ? hipStreamSynchronize(E->stream) : hipSuccess;
    release(E);
    if (e != hipSuccess) return fail(MECH_E_DEVICE, "stream synchronisation failed: %s", hipGetErrorString(e));
    return MECH_OK;
}

}  // extern "C"
