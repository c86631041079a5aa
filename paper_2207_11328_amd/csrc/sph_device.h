// Device-side helpers shared by the HIP translation units of libsph.so.
// gfx950 (CDNA4): wave64, 256 CUs in 8 XCDs, 160 KB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "sph.h"

namespace sph {

constexpr int kWave = 64;
constexpr uint32_t kTypeShift = 30;
constexpr uint32_t kBoundary = 1;
constexpr uint32_t kIndexMask = (1u << SPH_NEIB_INDEX_BITS) - 1u;

__device__ __forceinline__ uint32_t ptype(uint32_t info) { return info >> kTypeShift; }

// Linear cell index (relative to the scene's cell base) -> integer coordinates.
struct CellDims {
    int nx, ny, nz;
    uint32_t periodic;
};

__device__ __forceinline__ void cell_coords(int lc, const CellDims &d, int &cx, int &cy, int &cz)
{
    cx = lc % d.nx;
    int t = lc / d.nx;
    cy = t % d.ny;
    cz = t / d.ny;
}

// Squared separation of the neighbour predicate, in float32 with every
// operation rounded separately (no contraction), so that the decision is
// reproducible bit for bit:  x_d = t2_d + (o_i,d - o_j,d),  r2 = (xx + yy) + zz.
__device__ __forceinline__ float predicate_r2(float oix, float oiy, float oiz, float ojx, float ojy,
                                              float ojz, float t2x, float t2y, float t2z)
{
#pragma clang fp contract(off)
    const float x = t2x + (oix - ojx);
    const float y = t2y + (oiy - ojy);
    const float z = t2z + (oiz - ojz);
    const float xx = x * x;
    const float yy = y * y;
    const float zz = z * z;
    const float s = xx + yy;
    return s + zz;
}

// k * cs for k in {-1, 0, 1}, exact.
__device__ __forceinline__ float cell_shift(int k, float cs)
{
    return k == 0 ? 0.0f : (k > 0 ? cs : -cs);
}

// Neighbour entry: sorted index plus k_d = c_i,d - c_j,d in {-1, 0, 1} per
// axis as two's-complement 2-bit fields at bits 26, 28, 30.
__device__ __forceinline__ uint32_t pack_neib(uint32_t j, int kx, int ky, int kz)
{
    return j | ((uint32_t)kx & 3u) << 26 | ((uint32_t)ky & 3u) << 28 | ((uint32_t)kz & 3u) << 30;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Cell difference k_d in {-1, 0, 1} of axis d, stored as a two's-complement
// 2-bit field at bit 26 + 2d of a list entry.
__device__ __forceinline__ float entry_k(uint32_t e, int axis)
{
    return (float)((int32_t)(e << (4 - 2 * axis)) >> 30);
}

// Storage slot of the k-th pair of a list with nf fluid entries (front) and
// the boundary ones (back), k clamped to last = count - 1.
__device__ __forceinline__ int list_slot(int k, int nf, int last, int M)
{
    const int kk = min(k, last);
    return kk < nf ? kk : M - 1 + nf - kk;
}

// ---------------------------------------------------------------------------
// Cell bricks: blocks of cells processed by one workgroup with the particles
// of the brick and of its one-cell halo staged in LDS (used by the list build
// and by the derivative kernel).
// Bricks of cells: the unit of LDS staging of the list build and of the
// derivative kernels.  The brick-local lists written by the build index the
// staging order of the same bricks, so the build and its consumers take the
// shape from the same grid description (sph_grid.brick).  Supported shapes,
// the first being the default (zero shape):
constexpr int kShapes = 3;
constexpr int kShapeTable[kShapes][3] = {{3, 4, 3}, {3, 3, 3}, {3, 2, 3}};

// index into kShapeTable of a grid's brick shape, -1 if unsupported
inline int brick_shape_index(const int32_t b[3])
{
    if (b[0] == 0 && b[1] == 0 && b[2] == 0) return 0;
    for (int k = 0; k < kShapes; ++k)
        if (b[0] == kShapeTable[k][0] && b[1] == kShapeTable[k][1] && b[2] == kShapeTable[k][2]) return k;
    return -1;
}

// Calls f.template operator()<BX, BY, BZ>() for the shape of index k.
template <typename F>
inline void with_shape(int k, F &&f)
{
    switch (k) {
    case 1: f.template operator()<3, 3, 3>(); break;
    case 2: f.template operator()<3, 2, 3>(); break;
    default: f.template operator()<3, 4, 3>(); break;
    }
}

// Threads of a workgroup for bricks of `cells` cells: one lane per central
// particle up to 27 per cell (the densest lattice alignment), in whole waves.
constexpr int brick_threads(int cells) { return ((27 * cells + 63) / 64) * 64 > 1024 ? 1024 : ((27 * cells + 63) / 64) * 64; }

// Staging geometry of a brick of BX x BY x BZ cells: the brick and its
// one-cell halo, SX x SY x SZ staged cells numbered x fastest, then z, then y
// (y outermost, so the staged cells of the lower and of the upper half of the
// brick's y extent are two contiguous ranges of the staging order).  Inner
// cells u = ix + BX (iz + BZ iy) follow the same order.
template <int BX, int BY, int BZ>
struct Staging {
    static constexpr int SX = BX + 2, SY = BY + 2, SZ = BZ + 2;
    static constexpr int S = SX * SY * SZ, NI = BX * BY * BZ;
    __host__ __device__ static int cell(int sx, int sy, int sz) { return sx + SX * (sz + SZ * sy); }
    __host__ __device__ static int sx_of(int t) { return t % SX; }
    __host__ __device__ static int sz_of(int t) { return (t / SX) % SZ; }
    __host__ __device__ static int sy_of(int t) { return t / (SX * SZ); }
    __host__ __device__ static int ix_of(int u) { return u % BX; }
    __host__ __device__ static int iz_of(int u) { return (u / BX) % BZ; }
    __host__ __device__ static int iy_of(int u) { return u / (BX * BZ); }
    // staged cell of inner cell u, and the step to a neighbour cell
    __host__ __device__ static int inner(int u) { return cell(ix_of(u) + 1, iy_of(u) + 1, iz_of(u) + 1); }
    __host__ __device__ static int step(int dx, int dy, int dz) { return dx + SX * (dz + SZ * dy); }
};

// Brick-local lists: uint16 entries in groups of 8 per particle (one 16-byte
// load), tiles of 64 particles, group-major inside a tile: entry p of
// particle i is at brick_entry(i, p, groups), groups = ceil(max_neibs / 8).
constexpr int kBrickGroup = 8;
__host__ __device__ inline int brick_groups(int max_neibs) { return (max_neibs + kBrickGroup - 1) / kBrickGroup; }
__host__ __device__ inline size_t brick_entry(int i, int p, int groups)
{
    return ((size_t)(i / kWave) * groups + (size_t)(p / kBrickGroup)) * (kWave * kBrickGroup) +
           (size_t)(i % kWave) * kBrickGroup + (size_t)(p % kBrickGroup);
}

// Table of the bricks with a pair, written by the list build behind the
// brick-local lists of the same array (4-byte aligned: the lists take a
// multiple of 512 entries): int32 words [0] heavy bricks, [1 .. capacity]
// brick ids, heavy ones from the front and light ones from the back
// (brick_at), [capacity + 1] light bricks, [capacity + 2 ..] reserved.  A
// brick has a pair when one of its inner cells holds a particle with a
// non-empty list; at most one brick per such particle, so capacity ids
// suffice.
__host__ __device__ inline size_t brick_list_entries(int capacity, int max_neibs)
{
    return (size_t)((capacity + kWave - 1) / kWave) * kWave * (size_t)brick_groups(max_neibs) * kBrickGroup;
}
__host__ __device__ inline size_t brick_table_words(int capacity) { return (size_t)(capacity > 0 ? capacity : 1) + 4; }
__host__ __device__ inline int brick_table_cap(int capacity) { return capacity > 0 ? capacity : 1; }
template <typename T>
__host__ __device__ inline T *brick_table(T *neibs_brick, int capacity, int max_neibs)
{
    return (T *)((uint16_t *)neibs_brick + brick_list_entries(capacity, max_neibs));
}

struct BrickGrid {
    int nx, ny, nz;
    uint32_t periodic;
    int nbx, nby, nbz;
};

template <int BX, int BY, int BZ>
inline BrickGrid brick_grid(const int32_t ncell[3], uint32_t periodic)
{
    BrickGrid G;
    G.nx = ncell[0];
    G.ny = ncell[1];
    G.nz = ncell[2];
    G.periodic = periodic;
    G.nbx = (G.nx + BX - 1) / BX;
    G.nby = (G.ny + BY - 1) / BY;
    G.nbz = (G.nz + BZ - 1) / BZ;
    return G;
}

// Entry s (0..7) of a 16-byte group of brick-local list entries.
__device__ __forceinline__ uint32_t group_entry(const uint4 &g, int s)
{
    const uint32_t w = (s >> 1) == 0 ? g.x : (s >> 1) == 1 ? g.y : (s >> 1) == 2 ? g.z : g.w;
    return (s & 1) ? (w >> 16) : (w & 0xFFFFu);
}

__device__ __forceinline__ bool wrap_axis(int &c, int n, uint32_t periodic)
{
    if (periodic) {
        if (c < 0) c += n;
        if (c >= n) c -= n;
        return true;
    }
    return c >= 0 && c < n;
}

// exclusive scan of one int per thread over a block of NT threads
template <int NT>
__device__ __forceinline__ int block_scan(int v, int &total, int *wsum)
{
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    int inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    int off = 0;
    total = 0;
#pragma unroll
    for (int k = 0; k < NT / kWave; ++k) {
        off += k < w ? wsum[k] : 0;
        total += wsum[k];
    }
    __syncthreads();
    return off + inc - v;
}

// List the bricks that hold at least one particle (order is irrelevant: each
// brick writes only its own particles).  active[0] must be zero on entry.
// With cell_flags (one byte per cell, set by the list build for every cell
// that holds a particle with a non-empty list), a brick is listed only if one
// of its inner cells is flagged: the kernels that take the list write the
// outputs of particles with empty lists without staging, so a brick of such
// particles (a wall away from the fluid) needs none.  The flags of the brick's inner cells are
// cleared for the next call; a stale flag only lists a brick that then finds
// no pair.
// With light (a second counter, zero on entry), bricks with fewer than
// light_min particles are listed from the back of the id region instead
// (active[cap_ids], active[cap_ids - 1], ...; light[0] of them), so that a
// consumer taking the bricks in brick_at order ends with the cheap ones.
template <int BX, int BY, int BZ>
__global__ __launch_bounds__(256) void k_active_bricks(const int32_t *__restrict__ cell_start,
                                                       const int32_t *__restrict__ cell_end, BrickGrid G,
                                                       int32_t *__restrict__ active, uint8_t *__restrict__ cell_flags,
                                                       int32_t *__restrict__ light = nullptr, int light_min = 0,
                                                       int cap_ids = 0)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    const int nb = G.nbx * G.nby * G.nbz;
    int cnt = 0;
    bool flagged = cell_flags == nullptr;
    if (b < nb) {
        const int cx0 = (b % G.nbx) * BX, cy0 = ((b / G.nbx) % G.nby) * BY, cz0 = (b / (G.nbx * G.nby)) * BZ;
        const int cx1 = min(cx0 + BX, G.nx) - 1;
        // every row's loads are independent: all issued first (rows past the
        // grid edge read a valid row), then masked and summed
        int e[BY * BZ], s0[BY * BZ];
#pragma unroll
        for (int k = 0; k < BY * BZ; ++k) {
            const int y = min(cy0 + k % BY, G.ny - 1), z = min(cz0 + k / BY, G.nz - 1);
            const int row = G.nx * (y + G.ny * z);
            e[k] = cell_end[row + cx1];
            s0[k] = cell_start[row + cx0];
        }
        if (cell_flags) {
            uint8_t f[BY * BZ][BX];
#pragma unroll
            for (int k = 0; k < BY * BZ; ++k) {
                const int y = min(cy0 + k % BY, G.ny - 1), z = min(cz0 + k / BY, G.nz - 1);
                const int row = G.nx * (y + G.ny * z);
#pragma unroll
                for (int x = 0; x < BX; ++x) f[k][x] = cell_flags[row + min(cx0 + x, cx1)];
            }
            int any = 0;
#pragma unroll
            for (int k = 0; k < BY * BZ; ++k) {
                const int y = cy0 + k % BY, z = cz0 + k / BY;
                const int row = G.nx * (y + G.ny * z);
#pragma unroll
                for (int x = 0; x < BX; ++x) {
                    const bool in = y < G.ny && z < G.nz && cx0 + x <= cx1;
                    if (in && f[k][x]) {
                        any = 1;
                        cell_flags[row + cx0 + x] = 0;
                    }
                }
            }
            flagged = any != 0;
        }
#pragma unroll
        for (int k = 0; k < BY * BZ; ++k)
            cnt += (cy0 + k % BY < G.ny && cz0 + k / BY < G.nz) ? e[k] - s0[k] : 0;
    }
    const bool has = cnt > 0 && flagged;
    const bool lt = has && light && cnt < light_min;
    // wave-aggregated appends
    const unsigned long long ballot = __ballot(has && !lt), lballot = __ballot(lt);
    const int lane = threadIdx.x % kWave;
    const unsigned long long below = (1ull << lane) - 1ull;
    int base = 0, lbase = 0;
    if (lane == 0 && ballot) base = atomicAdd(&active[0], (int)__popcll(ballot));
    if (lane == 0 && lballot) lbase = atomicAdd(light, (int)__popcll(lballot));
    base = __shfl(base, 0);
    lbase = __shfl(lbase, 0);
    if (has && !lt) active[1 + base + __popcll(ballot & below)] = b;
    if (lt) active[cap_ids - (lbase + __popcll(lballot & below))] = b;
}

// Bricks listed by k_active_bricks: their number, and the kb-th in the order
// heavy (from the front) then light (from the back).
__device__ __forceinline__ int bricks_listed(const int32_t *active, const int32_t *light)
{
    return active[0] + light[0];
}
__device__ __forceinline__ int brick_at(const int32_t *active, int cap_ids, int kb)
{
    const int nh = active[0];
    return kb < nh ? active[1 + kb] : active[cap_ids - (kb - nh)];
}

// The two speeds of the adaptive time step of one fluid particle: its sound
// speed c = c0 (rho/rho0)^3 (gamma = 7) and |a + g| from its derivatives,
// in float32 with a fixed operation order (every kernel that takes the
// step's maxima evaluates them with this one definition, so they agree bit
// for bit).
__device__ __forceinline__ void dt_speeds(float rho, float fx, float fy, float fz, float rho0, float inv_rho0,
                                          float c0, float gx, float gy, float gz, float &c, float &a)
{
#pragma clang fp contract(off)
    const float d = (rho - rho0) * inv_rho0;
    const float b = 1.0f + d;
    c = c0 * b * b * b;
    const float x = fx + gx, y = fy + gy, z = fz + gz;
    a = __builtin_sqrtf(x * x + y * y + z * z);
}

// The adaptive step from the maxima of dt_speeds over the fluid particles
// (float32 maxima, taken to double): cfl min(h / c, sqrt(h / a)
// [, 0.125 h^2 / nu]); +inf scaled by cfl when nothing bounds it.
__device__ __forceinline__ double dt_from_maxima(double c, double a, double h, double nu, double cfl)
{
    double dt = INFINITY;
    if (c > 0.0) dt = h / c;
    if (a > 0.0) dt = fmin(dt, sqrt(h / a));
    if (nu > 0.0) dt = fmin(dt, 0.125 * h * h / nu);
    return cfl * dt;
}

// One stage of the explicit midpoint integrator for one particle (section
// "Code structure": predictor with dt/2, corrector with dt): the state (p, v)
// advances by tau along the stage velocity ua, the derivatives f plus gravity
// g and the density rate f.w; a boundary particle advances its density only.
// Every kernel that integrates goes through this one definition, so the
// fused and the separate forms of a stage agree bit for bit.
__device__ __forceinline__ void midpoint_stage(float4 &p, float4 &v, const float4 &ua, const float4 &f,
                                               bool boundary, float tau, float gx, float gy, float gz)
{
    if (!boundary) {
        p.x = fmaf(tau, ua.x, p.x);
        p.y = fmaf(tau, ua.y, p.y);
        p.z = fmaf(tau, ua.z, p.z);
        v.x = fmaf(tau, f.x + gx, v.x);
        v.y = fmaf(tau, f.y + gy, v.y);
        v.z = fmaf(tau, f.z + gz, v.z);
    }
    v.w = fmaf(tau, f.w, v.w);
}

// A counter zeroed by a kernel (graph-capturable, no memset node).
template <typename T>
__global__ void k_zero_one(T *p)
{
    *p = T(0);
}

}  // namespace sph

// Host-side launch helpers.
#define SPH_CHECK_LAUNCH()                                  \
    do {                                                    \
        if (hipGetLastError() != hipSuccess) return SPH_ERR_HIP; \
    } while (0)

// Compute units of the current device, queried once per device and kept
// (the only state the library holds between calls): persistent brick kernels
// launch one workgroup per CU.
static inline int sph_device_cus()
{
    static std::atomic<int> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int v = cus[dev].load(std::memory_order_relaxed);
    if (v <= 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cus[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

static inline unsigned sph_blocks(long long n, int threads)
{
    return (unsigned)((n + threads - 1) / threads);
}
