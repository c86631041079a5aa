// Neighbour search: re-bin, counting sort by cell with an in-cell sort by
// (type, id), reorder, cell ranges and split neighbour lists.
//
// Sort order is cell, then particle type, then particle id (section
// "Changing perspective: from the particle to the cell").  Instead of a
// multi-pass radix sort of 64-bit keys, the cell index is used directly as
// a single radix digit: a histogram over cells, an exclusive scan (which is
// also the cell-start array) and an atomic scatter put every particle in its
// cell's range; one wave per cell then ranks the cell's few particles by
// their (type, id) word, which makes the permutation unique.
//
// Lists are split (fluid from the front, boundary from the back) and stored
// neighbour-major (section "Efficient split neighbors list").
#include <hip/hip_runtime.h>

#include "sph_device.h"

using namespace sph;

namespace {

constexpr int kThreads = 256;
constexpr int kScanItems = 4;                       // per thread
constexpr int kScanTile = kThreads * kScanItems;    // elements per block

struct BuildLayout {
    size_t cnt, cursor, start, partials, perm_a, perm_b, t_cell, t_pos, t_vel, t_info, active, flags, total;
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

BuildLayout build_layout(int64_t capacity, int64_t n_cells)
{
    const int64_t nb = n_cells + 1;  // one extra bucket for dropped particles
    const int64_t nparts = (nb + kScanTile - 1) / kScanTile;
    BuildLayout L;
    size_t o = 0;
    L.cnt = o;      o = align_up(o + sizeof(int32_t) * nb);
    L.cursor = o;   o = align_up(o + sizeof(int32_t) * nb);
    L.start = o;    o = align_up(o + sizeof(int32_t) * (nb + 1));
    L.partials = o; o = align_up(o + sizeof(int32_t) * (nparts + 1));
    L.perm_a = o;   o = align_up(o + sizeof(uint32_t) * capacity);
    L.perm_b = o;   o = align_up(o + sizeof(uint32_t) * capacity);
    L.t_cell = o;   o = align_up(o + sizeof(int32_t) * capacity);
    L.t_pos = o;    o = align_up(o + sizeof(float4) * capacity);
    L.t_vel = o;    o = align_up(o + sizeof(float4) * capacity);
    L.t_info = o;   o = align_up(o + sizeof(uint32_t) * capacity);
    L.active = o;   o = align_up(o + sizeof(int32_t) * (n_cells + 1));
    L.flags = o;    o = align_up(o + (size_t)n_cells + 4);
    L.total = o;
    return L;
}

// Everything the build counts into starts at zero, in one launch (a kernel,
// not a memset, so that a captured graph holds no memset node): the bucket
// counts and cursors (nb each), the status words, the cell flags of the
// table of bricks with a pair (flag_words int32 words, none without brick
// lists) and the counters of the active-brick list and of that table.
__global__ void k_build_zero(int64_t nb, int32_t *__restrict__ cnt, int32_t *__restrict__ cursor,
                             int32_t *__restrict__ status, int64_t flag_words, int32_t *__restrict__ flags,
                             int32_t *__restrict__ active, int32_t *__restrict__ table_heavy,
                             int32_t *__restrict__ table_light)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = t; i < nb; i += stride) {
        cnt[i] = 0;
        cursor[i] = 0;
    }
    for (int64_t i = t; i < flag_words; i += stride) flags[i] = 0;
    if (t < SPH_STATUS_WORDS) status[t] = 0;
    if (t == 0) {
        *active = 0;
        if (table_heavy) {
            *table_heavy = 0;
            *table_light = 0;
        }
    }
}

// atomicAdd(&cnt[key], 1) for every valid lane of a wave, combined over runs
// of consecutive lanes with the same key (particles come in the order of the
// last build, sorted by cell, so a run is typically a whole cell's part of
// the wave): one atomic per run.  Returns the value the lane's own atomic
// could have returned (the run's base plus the lane's rank in the run).
// Every lane of the wave must call it.
__device__ __forceinline__ int run_atomic_inc(int32_t *cnt, int key, bool valid)
{
    const int lane = threadIdx.x % kWave;
    const int prev = __shfl(key, lane > 0 ? lane - 1 : 0);
    const unsigned long long vmask = __ballot(valid);
    const bool prev_valid = lane > 0 && ((vmask >> (lane - 1)) & 1ull);
    const bool first = valid && (!prev_valid || prev != key);
    // run boundaries: run starts and invalid lanes
    const unsigned long long bounds = __ballot(first) | ~vmask;
    const unsigned long long upto = bounds & (~0ull >> (kWave - 1 - lane));  // bits <= lane
    const int rs = kWave - 1 - __clzll(upto | 1ull);
    const unsigned long long above = lane == kWave - 1 ? 0ull : bounds & (~0ull << (lane + 1));
    const int re = above ? __ffsll((long long)above) - 1 : kWave;
    int base = 0;
    if (first) base = atomicAdd(&cnt[key], re - rs);
    base = __shfl(base, rs);
    return base + (lane - rs);
}

// Re-bin offsets into [-cs/2, cs/2) (float32, at most 4 cells per axis) and
// count particles per cell.  Particles that leave a non-periodic axis, or
// whose offsets are not finite, become dropped (cell = -1, last bucket).
__global__ __launch_bounds__(kThreads) void k_rebin_count(
    int n, int32_t *__restrict__ cell, float4 *__restrict__ pos, CellDims dims, float csx, float csy,
    float csz, int cell_base, int n_cells, int32_t *__restrict__ cnt)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    const bool valid = i < n;
    int c = valid ? cell[i] : -1;
    int bucket = n_cells;
    if (valid && c >= 0) {
        int cc[3];
        cell_coords(c - cell_base, dims, cc[0], cc[1], cc[2]);
        float4 p = pos[i];
        float o[3] = {p.x, p.y, p.z};
        const float cs[3] = {csx, csy, csz};
        const int nd[3] = {dims.nx, dims.ny, dims.nz};
        bool ok = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const float half = 0.5f * cs[d];
            float v = o[d];
            for (int it = 0; it < 4; ++it) {
                if (v >= half) { v = v - cs[d]; cc[d] += 1; }
                else if (v < -half) { v = v + cs[d]; cc[d] -= 1; }
                else break;
            }
            if (!(v >= -half && v < half)) ok = false;
            if ((dims.periodic >> d) & 1u) {
                cc[d] %= nd[d];
                if (cc[d] < 0) cc[d] += nd[d];
            } else if (cc[d] < 0 || cc[d] >= nd[d]) {
                ok = false;
            }
            o[d] = v;
        }
        pos[i] = make_float4(o[0], o[1], o[2], p.w);
        if (ok) {
            const int lc = cc[0] + dims.nx * (cc[1] + dims.ny * cc[2]);
            cell[i] = lc + cell_base;
            bucket = lc;
        } else {
            cell[i] = -1;
        }
    }
    run_atomic_inc(cnt, bucket, valid);
}

// ---- exclusive scan of cnt[0..m) into start[0..m], start[m] = total --------
__device__ __forceinline__ int block_exclusive_scan(int v, int &total)
{
    __shared__ int wsum[kThreads / kWave];
    const int lane = threadIdx.x % kWave;
    const int w = threadIdx.x / kWave;
    int inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    int off = 0;
    total = 0;
#pragma unroll
    for (int k = 0; k < kThreads / kWave; ++k) {
        if (k < w) off += wsum[k];
        total += wsum[k];
    }
    __syncthreads();
    return off + inc - v;
}

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const int32_t *__restrict__ in, int m,
                                                          int32_t *__restrict__ partials)
{
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < m) s += in[base + k];
    int total;
    (void)block_exclusive_scan(s, total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void k_scan_partials(int32_t *__restrict__ partials, int np,
                                                            int32_t *__restrict__ grand_total)
{
    int carry = 0;
    for (int base = 0; base < np; base += kThreads) {
        const int i = base + threadIdx.x;
        const int v = i < np ? partials[i] : 0;
        int total;
        const int ex = block_exclusive_scan(v, total);
        if (i < np) partials[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) *grand_total = carry;
}

__global__ __launch_bounds__(kThreads) void k_scan_apply(const int32_t *__restrict__ in, int m,
                                                         const int32_t *__restrict__ partials,
                                                         int32_t *__restrict__ out)
{
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < m ? in[base + k] : 0;
        s += v[k];
    }
    int total;
    int ex = block_exclusive_scan(s, total) + partials[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < m) out[base + k] = ex;
        ex += v[k];
    }
}

// Place every particle in its bucket's range (order inside a bucket is
// arbitrary at this point).
__global__ __launch_bounds__(kThreads) void k_scatter(int n, const int32_t *__restrict__ cell,
                                                      int cell_base, int n_cells,
                                                      const int32_t *__restrict__ start,
                                                      int32_t *__restrict__ cursor,
                                                      uint32_t *__restrict__ perm)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    const bool valid = i < n;
    const int c = valid ? cell[i] : -1;
    const int b = c >= 0 ? c - cell_base : n_cells;
    const int r = run_atomic_inc(cursor, b, valid);
    if (valid) perm[start[b] + r] = (uint32_t)i;
}

// Rank each particle of a bucket by its info word (type << 30 | id) and
// write it to its final position.  Ids are unique; equal words (invalid
// input) are ranked by their slot so the result is a permutation in every
// case.  One wave per window of kWave consecutive positions of the scattered
// order (which is grouped by bucket): the wave ranks the buckets that start
// in its window, one after the other.  Most buckets of a grid can be empty
// (the air above a dam break); waves over positions visit only buckets that
// hold particles, where a wave per bucket would be dispatched for each.
__global__ __launch_bounds__(kThreads) void k_cell_sort(int n, const int32_t *__restrict__ cell, int cell_base,
                                                        int n_cells, const int32_t *__restrict__ start,
                                                        const uint32_t *__restrict__ perm_in,
                                                        const uint32_t *__restrict__ info,
                                                        uint32_t *__restrict__ perm_out)
{
    const int w0 = (blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave) * kWave;
    if (w0 >= n) return;  // uniform
    const int lane = threadIdx.x % kWave;
    const int p = w0 + lane;
    int b = 0;  // bucket of position p
    bool first = false;
    if (p < n) {
        const int c = cell[perm_in[p]];
        b = c >= 0 ? c - cell_base : n_cells;
        first = start[b] == p;
    }
    unsigned long long F = __ballot(first);
    while (F) {  // uniform: the buckets that start in the window
        const int k = __ffsll((long long)F) - 1;
        F &= F - 1;
        const int bk = __shfl(b, k);
        const int s = w0 + k;
        const int m = start[bk + 1] - s;
        for (int mb = 0; mb < m; mb += kWave) {
            const int me = mb + lane;
            const bool valid = me < m;
            const uint32_t idx = valid ? perm_in[s + me] : 0u;
            const uint32_t key = valid ? info[idx] : 0xFFFFFFFFu;
            int rank = 0;
            for (int tb = 0; tb < m; tb += kWave) {
                const int t = tb + lane;
                const uint32_t kt_lane = t < m ? info[perm_in[s + t]] : 0xFFFFFFFFu;
                const int cnt = min(kWave, m - tb);
                for (int u = 0; u < cnt; ++u) {
                    const uint32_t kt = __shfl(kt_lane, u);
                    rank += (kt < key || (kt == key && tb + u < me)) ? 1 : 0;
                }
            }
            if (valid) perm_out[s + rank] = idx;
        }
    }
}

// Reorder by the sort permutation.  Also counts the particles whose offset,
// mass, velocity or density is not finite (one atomic per wave), so that a
// state that blew up is reported by the build's status word.
__global__ __launch_bounds__(kThreads) void k_gather(int n, const uint32_t *__restrict__ perm,
                                                     const int32_t *__restrict__ cell,
                                                     const float4 *__restrict__ pos,
                                                     const float4 *__restrict__ vel,
                                                     const uint32_t *__restrict__ info,
                                                     int32_t *__restrict__ o_cell,
                                                     float4 *__restrict__ o_pos,
                                                     float4 *__restrict__ o_vel,
                                                     uint32_t *__restrict__ o_info,
                                                     uint32_t *__restrict__ perm_out,
                                                     int32_t *__restrict__ status)
{
    const int k = blockIdx.x * kThreads + threadIdx.x;
    bool bad = false;
    if (k < n) {
        const uint32_t src = perm[k];
        if (perm_out) perm_out[k] = src;
        const float4 p = pos[src];
        const float4 v = vel[src];
        o_cell[k] = cell[src];
        o_pos[k] = p;
        o_vel[k] = v;
        o_info[k] = info[src];
        bad = !(isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(p.w) && isfinite(v.x) &&
                isfinite(v.y) && isfinite(v.z) && isfinite(v.w));
    }
    const unsigned long long m = __ballot(bad);
    if (m && (threadIdx.x % kWave) == 0) atomicAdd(&status[SPH_STATUS_NONFINITE], (int)__popcll(m));
}

// The sorted state back into the caller's arrays.  Also: particles dropped
// by the build are in no brick and get no neighbours (count 0), and, when
// flags is not null, the cells that hold a particle with a non-empty list
// are flagged (for the table of bricks with a pair).
__global__ __launch_bounds__(kThreads) void k_copy_state(int n, const int32_t *__restrict__ cell,
                                                         const float4 *__restrict__ pos,
                                                         const float4 *__restrict__ vel,
                                                         const uint32_t *__restrict__ info,
                                                         int32_t *__restrict__ o_cell,
                                                         float4 *__restrict__ o_pos,
                                                         float4 *__restrict__ o_vel,
                                                         uint32_t *__restrict__ o_info,
                                                         uint32_t *__restrict__ neib_count, int cell_base,
                                                         int n_cells, uint8_t *__restrict__ flags)
{
    const int k = blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    const int c = cell[k];
    o_cell[k] = c;
    o_pos[k] = pos[k];
    o_vel[k] = vel[k];
    o_info[k] = info[k];
    if (c < 0) {
        neib_count[k] = 0u;
    } else if (flags && neib_count[k] != 0u) {
        const int lc = c - cell_base;
        if ((unsigned)lc < (unsigned)n_cells) flags[lc] = 1;
    }
}

// Cell ranges from the bucket starts; thread 0 also writes the particles in
// cells and the dropped ones (the last bucket) to the status words.
__global__ __launch_bounds__(kThreads) void k_cell_ranges(int n_cells, const int32_t *__restrict__ start,
                                                          int32_t *__restrict__ cell_start,
                                                          int32_t *__restrict__ cell_end, int n,
                                                          int32_t *__restrict__ status)
{
    const int c = blockIdx.x * kThreads + threadIdx.x;
    if (c == 0) {
        const int n_active = start[n_cells];
        status[SPH_STATUS_N_ACTIVE] = n_active;
        status[SPH_STATUS_DROPPED] = n - n_active;
    }
    if (c >= n_cells) return;
    cell_start[c] = start[c];
    cell_end[c] = start[c + 1];
}

// Neighbour lists, cell-brick form (section "Changing perspective: from the
// particle to the cell": a group of work-items per cell, neighbour data shared
// through on-chip memory).  A workgroup owns a brick of BX x BY x BZ cells and
// stages the offsets and type words of the particles of the brick and its
// one-cell halo in LDS (16 bytes per particle).  Each lane then takes one
// central particle and scans the 27 cells of its Moore neighbourhood (z, y, x
// from -1 to +1), each cell in sorted order, reading candidates from LDS;
// lanes of the same cell read the same candidate at the same time (an LDS
// broadcast).  Fluid entries fill the list from the front and boundary
// entries from the back, in scan order, until M entries are written.
//
// Inside a cell fluid particles precede boundary ones, so the exclusion of
// boundary-boundary pairs is a shorter candidate range for a boundary centre
// (the fluid prefix of each cell, from a per-cell table) rather than a test per
// candidate, and the candidate loop has no data-dependent branch: one
// predicated store per listed pair.  A brick whose halo does not fit in LDS
// runs the same loop on global memory.
//
// Optionally the same lists are also written in brick-local form for the
// derivative kernels: entry k is the neighbour's slot in the staging order of
// the central particle's brick (cells of the brick and its halo in the
// Staging order, particles of a cell in sorted order), uint16, in scan order with
// fluid and boundary neighbours interleaved as found (entries 0 .. nf+nb-1),
// stored in groups of 8 per particle (brick_entry).
// The staged word of a particle (w of its float4 in LDS): its type in the
// type bits, its staged cell in bits kCellShift.., and for a central the
// number of neighbours found so far in the low bits (kFoundMask; the count is
// below the brick's staged particles, fewer than kBuildCap).
constexpr uint32_t kFoundMask = 0xFFFFu;
constexpr int kCellShift = 16;
constexpr uint32_t kCellMask = 0xFFu;

// The split j-list of one central particle written from its brick-local
// list (w entries, already in global memory, in scan order), entry k of the
// lanes of a wave in one store.  The staged word of each entry's particle
// holds its staged cell t (kCellShift); the cell gives the particle index
// (slot - cDelta[t]) and, from the offset t - tc to the central's cell, the
// image code (sCode[t - tc + S - 1]).  Returns n_fluid | n_boundary << 16.
template <int BX, int BY, int BZ>
__device__ __forceinline__ uint32_t brick_jlists(int tc, int M, int w, const int *cDelta, const uint32_t *sCode,
                                                 const float4 *sPos, uint32_t *tile, const uint16_t *ltile)
{
    constexpr int S = Staging<BX, BY, BZ>::S;
    uint32_t *tf = tile, *tb = tile + (size_t)(M - 1) * kWave;
    const uint4 *lg = (const uint4 *)ltile;
    uint4 grp = make_uint4(0u, 0u, 0u, 0u);
    const uint32_t *code = sCode + (S - 1 - tc);
    for (int e = 0; e < w; ++e) {
        if ((e & (kBrickGroup - 1)) == 0) grp = lg[(size_t)(e / kBrickGroup) * kWave];
        const int word = e >> 1 & 3;
        const uint32_t pair = word == 0 ? grp.x : word == 1 ? grp.y : word == 2 ? grp.z : grp.w;
        const int sl = (int)(pair >> ((e & 1) * 16) & 0xFFFFu);
        const uint32_t ws = __float_as_uint(sPos[sl].w);
        const int t = (int)(ws >> kCellShift & kCellMask);
        const bool nb_boundary = ptype(ws) == kBoundary;
        *(nb_boundary ? tb : tf) = (uint32_t)(sl - cDelta[t]) | code[t];
        tf += nb_boundary ? 0 : kWave;
        tb -= nb_boundary ? kWave : 0;
    }
    const int wf = (int)((tf - tile) / kWave), wb = w - wf;
    return (uint32_t)wf | (uint32_t)wb << 16;
}

template <int BX, int BY, int BZ, bool LDS>
__device__ __forceinline__ uint32_t brick_scan(int i, int tc, int M, const float4 &pi, bool central_boundary,
                                               const int *cBase, const int *cDelta, const int *cFluidEnd,
                                               const float4 *sPos, const float4 *__restrict__ gpos,
                                               const uint32_t *__restrict__ ginfo, float csx, float csy, float csz,
                                               float rs2, uint32_t *tile, uint16_t *ltile, int &total_found)
{
    // Each neighbour cell is scanned in chunks of up to 64 candidates in two
    // phases: the predicate alone, one bit per hit in a 64-bit mask, then the
    // hits in slot order, written as before.  Only about one candidate in six
    // is a hit, so the writing work runs per hit instead of per candidate.
    int found = 0, w = 0;
    // write positions: the next fluid slot from the front, the next boundary
    // slot from the back; the brick-local entries of the current group of 8
    // are collected in registers and stored as one 16-byte group when it is
    // full (groups are kWave x 8 entries apart), the last one at the end.
    // (With the brick staged in LDS and brick-local lists asked for, the
    // cell form of the scan runs instead.)
    uint32_t *tf = tile, *tb = tile + (size_t)(M - 1) * kWave;
    uint4 *lg = (uint4 *)ltile;
    uint4 grp = make_uint4(0u, 0u, 0u, 0u);
    for (int dz = -1; dz <= 1; ++dz) {
        const float t2z = cell_shift(-dz, csz);
        for (int dy = -1; dy <= 1; ++dy) {
            const float t2y = cell_shift(-dy, csy);
            for (int dx = -1; dx <= 1; ++dx) {
                const float t2x = cell_shift(-dx, csx);
                const int t = tc + Staging<BX, BY, BZ>::step(dx, dy, dz);
                const int s0 = cBase[t];
                const int s1 = central_boundary ? cFluidEnd[t] : cBase[t + 1];
                const int delta = cDelta[t];
                const uint32_t code = pack_neib(0u, -dx, -dy, -dz);
                // the central itself can only be met in its own cell (the 27
                // cells are distinct grid cells), at slot i + delta there
                const int self_sl = (dx | dy | dz) == 0 ? i + delta : -1;
                for (int c0 = s0; c0 < s1; c0 += 64) {
                    const int m = min(s1 - c0, 64);
                    // hit bits of the chunk, candidates 0..31 and 32..63 in a
                    // 32-bit word each (the bit of candidate k is uniform)
                    uint32_t hlo = 0u, hhi = 0u;
                    // two candidates in flight per lane (the LDS read latency)
#pragma unroll 2
                    for (int k = 0; k < min(m, 32); ++k) {
                        const int sl = c0 + k;
                        const float4 pj = LDS ? sPos[sl] : gpos[sl - delta];
                        const float r2 = predicate_r2(pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, t2x, t2y, t2z);
                        hlo = r2 < rs2 ? hlo | 1u << k : hlo;
                    }
#pragma unroll 2
                    for (int k = 32; k < m; ++k) {
                        const int sl = c0 + k;
                        const float4 pj = LDS ? sPos[sl] : gpos[sl - delta];
                        const float r2 = predicate_r2(pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, t2x, t2y, t2z);
                        hhi = r2 < rs2 ? hhi | 1u << (k - 32) : hhi;
                    }
                    uint64_t hits = (uint64_t)hhi << 32 | hlo;
                    const int sk = self_sl - c0;
                    if ((unsigned)sk < 64u) hits &= ~(1ull << sk);
                    found += __popcll(hits);
                    while (hits) {
                        const int k = __ffsll((long long)hits) - 1;
                        hits &= hits - 1;
                        if (w < M) {
                            const int sl = c0 + k;
                            const int j = sl - delta;
                            {
                                const uint32_t inf = LDS ? __float_as_uint(sPos[sl].w) : ginfo[j];
                                const bool nb_boundary = ptype(inf) == kBoundary;
                                *(nb_boundary ? tb : tf) = (uint32_t)j | code;
                                tf += nb_boundary ? 0 : kWave;
                                tb -= nb_boundary ? kWave : 0;
                            }
                            if (ltile) {
                                const int e = w & (kBrickGroup - 1);
                                const uint32_t v = (uint32_t)min(sl, 0xFFFF) << ((e & 1) * 16);
                                grp.x |= (e >> 1) == 0 ? v : 0u;
                                grp.y |= (e >> 1) == 1 ? v : 0u;
                                grp.z |= (e >> 1) == 2 ? v : 0u;
                                grp.w |= (e >> 1) == 3 ? v : 0u;
                                if (e == kBrickGroup - 1) {
                                    lg[(size_t)(w / kBrickGroup) * kWave] = grp;
                                    grp = make_uint4(0u, 0u, 0u, 0u);
                                }
                            }
                            ++w;
                        }
                    }
                }
            }
        }
    }
    if (ltile && (w & (kBrickGroup - 1)) != 0) lg[(size_t)(w / kBrickGroup) * kWave] = grp;
    const int wf = (int)((tf - tile) / kWave), wb = w - wf;
    total_found = found;
    return (uint32_t)wf | (uint32_t)wb << 16;
}

// Scan of the list build, cell form (brick staged in LDS, brick-local lists
// asked for).  The work items are the kItemParts parts of each inner cell's
// central particles (consecutive runs); a wave takes items from a counter.  For its item, the
// wave lays the candidates of the cell's 27 neighbour cells, in scan order
// (cells z, y, x from -1 to +1, each in slot order; only the fluid prefix of
// each cell when the item's centrals are boundary particles), out over its
// lanes in chunks of 64, one candidate per lane with its cell shift, and
// tests every central of the item against each chunk: every lane busy on the
// same central, no divergent trip counts.  The hits of a chunk are a ballot;
// a hit's place in the central's list is the count of hits before it
// (mbcnt), so the entries come out in scan order and the first max_neibs
// found are kept, as in the lane-per-central form.  The brick-local entries
// go straight to global memory (the groups of one central fill within the
// item); the number found is kept in the low 30 bits of the central's staged
// type word (its type bits stay: other waves read them); a candidate past
// the cell set points at a dummy staged particle far away.
constexpr int kItemChunks = 6;                 // candidate chunks held in registers per pass
constexpr int kItemParts = 1;                  // work items per inner cell (its centrals split evenly)

// Tests of one central (LDS slot si, position pi) against the nch candidate
// chunks of the item; found: entries so far.  MASK_B: the central is a
// boundary particle among fluid candidates (boundary candidates are skipped).
// The hit mask of a chunk is formed from ballots of plain compares combined on
// the scalar unit (a ballot of a combined lane predicate would first be turned
// into a vector of 0/1 and compared again); a hit's entry is stored at its
// byte offset from the central's (uniform) group base.
template <bool MASK_B>
__device__ __forceinline__ int scan_central(int found, uint32_t si, const float4 &pi, int nch, const int *sa,
                                            const float *tx, const float *ty, const float *tz, const float4 *sPos,
                                            float rs2, int M, uint16_t *__restrict__ lt)
{
#pragma unroll
    for (int c = 0; c < kItemChunks; ++c) {
        if (c < nch) {  // uniform (scalar)
            const uint32_t slot = (uint32_t)sa[c];
            const float4 pj = sPos[slot];
            const float r2 = predicate_r2(pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, tx[c], ty[c], tz[c]);
            const bool in = r2 < rs2, other = slot != si;
            unsigned long long H = __builtin_amdgcn_ballot_w64(in) & __builtin_amdgcn_ballot_w64(other);
            bool fluid = true;
            if constexpr (MASK_B) {
                fluid = ptype(__float_as_uint(pj.w)) != kBoundary;
                H &= __builtin_amdgcn_ballot_w64(fluid);
            }
            if (H) {  // uniform
                const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(H >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)H, (uint32_t)found));
                // brick_entry layout: group pos / 8 at 1024-byte stride, entry pos % 8
                const uint32_t boff = ((pos >> 3) << 10) | ((pos & 7u) << 1);
                if (in && other && fluid && pos < (uint32_t)M)
                    *reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(lt) + boff) = (uint16_t)slot;
                found += (int)__popcll(H);
            }
        }
    }
    return found;
}

template <int BX, int BY, int BZ>
__device__ __forceinline__ void brick_scan_items(int M, int *sItem, const int *cBase, const int *cDelta,
                                                 const int *cFluidEnd, const int *iBase, const int *iStart,
                                                 float4 *sPos, int dummy_slot, float csx, float csy, float csz,
                                                 float rs2, uint16_t *__restrict__ neibs_brick)
{
    using St = Staging<BX, BY, BZ>;
    constexpr int NI = St::NI;
    const int lane = threadIdx.x % kWave;
    const int G = brick_groups(M);
    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(sItem, 1);
        item = __builtin_amdgcn_readfirstlane(__shfl(item, 0));
        if (item >= kItemParts * NI) break;  // uniform
        const int u = item / kItemParts, part = item % kItemParts;
        const int n_u = iBase[u + 1] - iBase[u];
        const int qa = part * n_u / kItemParts, qb = (part + 1) * n_u / kItemParts;
        if (qa >= qb) continue;  // uniform
        const int tc = St::inner(u);
        const int i0 = iStart[u];
        const int sdel = cDelta[tc];
        // centrals are fluid first: a boundary one first means all are
        const bool fluid_only = ptype(__float_as_uint(sPos[i0 + qa + sdel].w)) == kBoundary;
        // candidate ranges of the 27 cells, lane k < 27 (k = 9 (dz+1) + 3 (dy+1) + dx+1)
        int beg = 0, len = 0;
        if (lane < 27) {
            const int t = tc + St::step(lane % 3 - 1, (lane / 3) % 3 - 1, lane / 9 - 1);
            beg = cBase[t];
            len = (fluid_only ? cFluidEnd[t] : cBase[t + 1]) - beg;
        }
        // inclusive scan over lanes 0..26; the lane id is read afresh (opaque
        // to the compiler) so that the shuffle addresses are not kept live
        // across the whole item loop
        int incl = len, me;
        asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0" : "=v"(me));
#pragma unroll
        for (int o = 1; o < 32; o <<= 1) {
            const int v = __builtin_amdgcn_ds_bpermute((me - o) << 2, incl);
            if (me >= o) incl += v;
        }
        const int ex = incl - len;
        const int ncand = __builtin_amdgcn_readfirstlane(__shfl(incl, 26));
        if (ncand == 0) {  // uniform: no candidate (boundary centrals far from the fluid)
            for (int q = qa + lane; q < qb; q += kWave) {
                uint32_t *wq = reinterpret_cast<uint32_t *>(&sPos[i0 + q + sdel]) + 3;
                *wq &= ~kFoundMask;
            }
            continue;
        }
        for (int pg = 0; pg < ncand; pg += kItemChunks * kWave) {
            int sa[kItemChunks];
            float tx[kItemChunks], ty[kItemChunks], tz[kItemChunks];
#pragma unroll
            for (int c = 0; c < kItemChunks; ++c) {
                const int idx = pg + c * kWave + lane;
                int lo = 0, hi = 26;  // the last cell k with ex_k <= idx
#pragma unroll
                for (int st = 0; st < 5; ++st) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (__shfl(ex, mid) <= idx) lo = mid;
                    else hi = mid - 1;
                }
                const int b = __shfl(beg, lo), e = __shfl(ex, lo);
                sa[c] = idx < ncand ? b + (idx - e) : dummy_slot;
                // k_d = c_i - c_j = -(d) for the neighbour cell at offset d
                tx[c] = cell_shift(1 - lo % 3, csx);
                ty[c] = cell_shift(1 - (lo / 3) % 3, csy);
                tz[c] = cell_shift(1 - lo / 9, csz);
            }
            const int nch = min(kItemChunks, (ncand - pg + kWave - 1) / kWave);
            const bool last_page = pg + kItemChunks * kWave >= ncand;
            for (int q = qa; q < qb; ++q) {  // uniform
                const int i = __builtin_amdgcn_readfirstlane(i0 + q), si = i + sdel;
                const float4 pi = sPos[si];
                const uint32_t wi = __builtin_amdgcn_readfirstlane(__float_as_uint(pi.w));
                int found = pg == 0 ? 0 : (int)(wi & kFoundMask);
                uint16_t *lt = neibs_brick + brick_entry(i, 0, G);
                // a boundary central among fluid ones takes fluid neighbours only
                if (!fluid_only && ptype(wi) == kBoundary)
                    found = scan_central<true>(found, si, pi, nch, sa, tx, ty, tz, sPos, rs2, M, lt);
                else
                    found = scan_central<false>(found, si, pi, nch, sa, tx, ty, tz, sPos, rs2, M, lt);
                if (last_page) {
                    // zero the rest of the last group, so the lists are the same bytes
                    // whatever the array held
                    const int w = min(found, M);
                    const int wend = min((w + kBrickGroup - 1) & ~(kBrickGroup - 1), G * kBrickGroup);
                    const int e = w + lane;
                    if (e < wend) lt[((e >> 3) << 9) | (e & 7)] = 0;
                }
                if (lane == 0)
                    reinterpret_cast<uint32_t *>(&sPos[si])[3] =
                        (wi & ~kFoundMask) | (uint32_t)min(found, (int)kFoundMask);
            }
        }
    }
}

template <int BX, int BY, int BZ, int NT, int CAP>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT / 128))) void k_build_brick(int n, int max_neibs, const float4 *__restrict__ pos,
                                                    const uint32_t *__restrict__ info,
                                                    const int32_t *__restrict__ start, BrickGrid G, float csx,
                                                    float csy, float csz, float rs2,
                                                    const int32_t *__restrict__ active,
                                                    uint32_t *__restrict__ neibs,
                                                    uint16_t *__restrict__ neibs_brick,
                                                    uint32_t *__restrict__ neib_count,
                                                    int32_t *__restrict__ status)
{
    constexpr int SX = BX + 2, SY = BY + 2, SZ = BZ + 2;
    constexpr int S = SX * SY * SZ;
    constexpr int NI = BX * BY * BZ;
    static_assert(S <= NT && NI <= NT, "one thread per cell");
    __shared__ float4 sPos[CAP];  // xyz offset, w = type/id word
    __shared__ int cBase[S + 1];
    __shared__ int cDelta[S];
    __shared__ int cFluidEnd[S];  // end of the fluid prefix of each staged cell (slot)
    __shared__ int iBase[NI + 1];
    __shared__ int iStart[NI];
    __shared__ int wsum[NT / kWave];
    __shared__ int sItem;  // work items taken (cell form of the scan)
    // image code of the neighbour cell at staged offset d = t - tc from the
    // central's cell, at index d + S - 1 (offsets that are no neighbour: 0)
    __shared__ uint32_t sCode[2 * S - 1];
    static_assert(S - 1 <= (int)kCellMask, "the staged cell fits its field of the staged word");

    const int tid = threadIdx.x;
    if ((int)blockIdx.x >= active[0]) return;
    for (int k = tid; k < 2 * S - 1; k += NT) {  // (read after the staging barrier)
        // d = dx + SX (dz + SZ dy) with dx, dy, dz in {-1, 0, 1}, d + S - 1 = k
        const int e = k - (S - 1) + 1 + SX + SX * SZ;
        const int ex = e % SX, ez = (e / SX) % SZ, ey = e / (SX * SZ);
        const bool nb = e >= 0 && ex <= 2 && ez <= 2 && ey <= 2;
        sCode[k] = nb ? pack_neib(0u, 1 - ex, 1 - ey, 1 - ez) : 0u;
    }
    const int b = active[1 + blockIdx.x];
    const int cx0 = (b % G.nbx) * BX, cy0 = ((b / G.nbx) % G.nby) * BY, cz0 = (b / (G.nbx * G.nby)) * BZ;

    // 1. ranges of the staged cells and their LDS bases
    int st = 0, cnt = 0;
    if (tid < S) {
        using St = Staging<BX, BY, BZ>;
        int gx = cx0 - 1 + St::sx_of(tid), gy = cy0 - 1 + St::sy_of(tid), gz = cz0 - 1 + St::sz_of(tid);
        const bool ok = wrap_axis(gx, G.nx, G.periodic & 1u) && wrap_axis(gy, G.ny, (G.periodic >> 1) & 1u) &&
                        wrap_axis(gz, G.nz, (G.periodic >> 2) & 1u);
        if (ok) {
            const int lin = gx + G.nx * (gy + G.ny * gz);
            st = start[lin];
            cnt = start[lin + 1] - st;
        }
    }
    int total;
    const int ex = block_scan<NT>(cnt, total, wsum);
    if (tid < S) {
        cBase[tid] = ex;
        cDelta[tid] = ex - st;
        cFluidEnd[tid] = ex + cnt;  // lowered below where the cell holds boundary particles
    }
    if (tid == 0) cBase[S] = total;
    __syncthreads();
    int icnt = 0, ist = 0;
    // inner cells past the grid edge hold no centrals (on a periodic axis the
    // staged copy would be the wrapped cell, owned by another brick)
    using St = Staging<BX, BY, BZ>;
    if (tid < NI && cx0 + St::ix_of(tid) < G.nx && cy0 + St::iy_of(tid) < G.ny && cz0 + St::iz_of(tid) < G.nz) {
        const int t = St::inner(tid);
        icnt = cBase[t + 1] - cBase[t];
        ist = cBase[t] - cDelta[t];
    }
    int nc;
    const int iex = block_scan<NT>(icnt, nc, wsum);
    if (tid < NI) {
        iBase[tid] = iex;
        iStart[tid] = ist;
    }
    if (tid == 0) iBase[NI] = nc;
    if (nc == 0) return;  // uniform: no particle in the brick
    // (one staged slot past the brick is the cell form's dummy candidate)
    const bool use_lds = total < CAP;
    // the cell form of the scan needs the brick-local lists (the j-lists are
    // written from them)
    const bool cells = use_lds && neibs_brick != nullptr;

    // 2. stage the brick and its halo (slot -> cell by binary search) and mark
    //    the first boundary particle of each cell
    for (int s2 = tid; s2 < total; s2 += NT) {
        int lo = 0, hi = S - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (cBase[mid] <= s2) lo = mid;
            else hi = mid - 1;
        }
        const int j = s2 - cDelta[lo];
        const uint32_t inf = info[j];
        if (use_lds) {
            float4 p = pos[j];
            p.w = __uint_as_float((inf & ~((1u << kTypeShift) - 1u)) | (uint32_t)lo << kCellShift);
            sPos[s2] = p;
        }
        if (ptype(inf) == kBoundary && (s2 == cBase[lo] || ptype(info[j - 1]) != kBoundary)) cFluidEnd[lo] = s2;
    }
    if (cells && tid == 0) {
        sPos[total] = make_float4(1e18f, 1e18f, 1e18f, 0.0f);  // no central is within r_s of it
        sItem = 0;
    }
    __syncthreads();

    if (cells) {
        // 3a. the cell form of the scan: brick-local lists and counts found
        brick_scan_items<BX, BY, BZ>(max_neibs, &sItem, cBase, cDelta, cFluidEnd, iBase, iStart, sPos, total, csx,
                                     csy, csz, rs2, neibs_brick);
        __syncthreads();
        // 3b. one lane per central: its j-list from its brick-local list
        for (int q0 = 0; q0 < nc; q0 += NT) {
            const int q = q0 + tid;
            if (q >= nc) break;
            int lo = 0, hi = NI - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (iBase[mid] <= q) lo = mid;
                else hi = mid - 1;
            }
            const int u = lo;
            const int i = iStart[u] + (q - iBase[u]);
            const int tc = St::inner(u);
            const int found = (int)(__float_as_uint(sPos[i + cDelta[tc]].w) & kFoundMask);
            const size_t toff = (size_t)(i / kWave) * kWave * max_neibs + (i % kWave);
            const uint32_t cw = brick_jlists<BX, BY, BZ>(tc, max_neibs, min(found, max_neibs), cDelta, sCode, sPos,
                                                         neibs + toff,
                                                         neibs_brick + brick_entry(i, 0, brick_groups(max_neibs)));
            neib_count[i] = cw;
            atomicMax(&status[SPH_STATUS_MAX_NEIBS], found);
            if (found > max_neibs) atomicAdd(&status[SPH_STATUS_OVERFLOW], 1);
        }
        return;
    }

    // 3. one lane per central particle of the brick
    for (int q0 = 0; q0 < nc; q0 += NT) {
        const int q = q0 + tid;
        if (q >= nc) break;
        int lo = 0, hi = NI - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (iBase[mid] <= q) lo = mid;
            else hi = mid - 1;
        }
        const int u = lo;
        const int i = iStart[u] + (q - iBase[u]);
        const int tc = St::inner(u);
        const float4 pi = pos[i];
        const bool central_boundary = ptype(info[i]) == kBoundary;
        const size_t toff = (size_t)(i / kWave) * kWave * max_neibs + (i % kWave);
        uint32_t *tile = neibs + toff;
        uint16_t *ltile = neibs_brick ? neibs_brick + brick_entry(i, 0, brick_groups(max_neibs)) : nullptr;
        int found;
        const uint32_t cw =
            use_lds ? brick_scan<BX, BY, BZ, true>(i, tc, max_neibs, pi, central_boundary, cBase, cDelta, cFluidEnd,
                                                   sPos, pos, info, csx, csy, csz, rs2, tile, ltile, found)
                    : brick_scan<BX, BY, BZ, false>(i, tc, max_neibs, pi, central_boundary, cBase, cDelta,
                                                    cFluidEnd, sPos, pos, info, csx, csy, csz, rs2, tile, ltile,
                                                    found);
        neib_count[i] = cw;
        atomicMax(&status[SPH_STATUS_MAX_NEIBS], found);
        if (found > max_neibs) atomicAdd(&status[SPH_STATUS_OVERFLOW], 1);
    }
}

constexpr int kBuildCap = 4800;  // 75 KB of LDS for the halo: two workgroups per CU
static_assert(kBuildCap <= (int)kFoundMask, "a central's count of found neighbours fits its field");

bool grid_ok(const sph_grid *g, float r_search)
{
    for (int d = 0; d < 3; ++d) {
        if (g->ncell[d] < 1) return false;
        if (!(g->cell_size[d] >= r_search)) return false;
        if (((g->periodic >> d) & 1u) && g->ncell[d] < 3) return false;
    }
    const int64_t nc = (int64_t)g->ncell[0] * g->ncell[1] * g->ncell[2];
    if (nc + 2 > INT32_MAX || g->cell_base < 0 || nc + g->cell_base > INT32_MAX) return false;
    return true;
}

}  // namespace

extern "C" size_t sph_neib_list_entries(int32_t capacity, int32_t max_neibs)
{
    if (capacity < 0 || max_neibs < 0) return 0;
    return (size_t)((capacity + kWave - 1) / kWave) * kWave * (size_t)max_neibs;
}

extern "C" size_t sph_neib_brick_entries(int32_t capacity, int32_t max_neibs)
{
    if (capacity < 0 || max_neibs < 0) return 0;
    // the lists, then the table of bricks with a pair (int32 words)
    return brick_list_entries(capacity, max_neibs) + 2 * brick_table_words(capacity);
}

extern "C" size_t sph_build_workspace_bytes(int32_t capacity, int32_t n_cells)
{
    if (capacity < 0 || n_cells < 0) return 0;
    return build_layout(capacity, n_cells).total;
}

extern "C" int32_t sph_brick_shapes(int32_t *shapes, int32_t max_shapes)
{
    if (shapes)
        for (int k = 0; k < kShapes && k < max_shapes; ++k)
            for (int d = 0; d < 3; ++d) shapes[3 * k + d] = kShapeTable[k][d];
    return kShapes;
}

extern "C" sph_status sph_build_neighbors(const sph_grid *grid, const sph_params *params,
                                          sph_particles *parts, uint32_t *neibs, uint32_t *neib_count,
                                          int32_t max_neibs, int32_t *cell_start, int32_t *cell_end,
                                          int32_t *d_status, uint32_t *perm_out, uint16_t *neibs_brick,
                                          void *workspace, size_t workspace_bytes, void *stream)
{
    if (!grid || !params || !parts || !neibs || !neib_count || !cell_start || !cell_end || !d_status)
        return SPH_ERR_ARG;
    if (parts->n < 0 || parts->capacity < parts->n || parts->capacity > SPH_MAX_CAPACITY) return SPH_ERR_ARG;
    if (parts->capacity > 0 && (!parts->cell || !parts->pos || !parts->vel || !parts->info)) return SPH_ERR_ARG;
    if (max_neibs < 1 || max_neibs > 65535) return SPH_ERR_ARG;
    if (neibs_brick && ((uintptr_t)neibs_brick & 15u)) return SPH_ERR_ARG;  // written in 16-byte groups
    if (!(params->r_search > 0.0f) || !grid_ok(grid, params->r_search)) return SPH_ERR_ARG;
    const int shape = brick_shape_index(grid->brick);
    if (shape < 0) return SPH_ERR_ARG;
    const int n = parts->n;
    const int cap = parts->capacity;
    const int n_cells = grid->ncell[0] * grid->ncell[1] * grid->ncell[2];
    const BuildLayout L = build_layout(cap, n_cells);
    if (!workspace || workspace_bytes < L.total) return SPH_ERR_WORKSPACE;

    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    int32_t *cnt = (int32_t *)(ws + L.cnt);
    int32_t *cursor = (int32_t *)(ws + L.cursor);
    int32_t *start = (int32_t *)(ws + L.start);
    int32_t *partials = (int32_t *)(ws + L.partials);
    uint32_t *perm_a = (uint32_t *)(ws + L.perm_a);
    uint32_t *perm_b = (uint32_t *)(ws + L.perm_b);
    int32_t *t_cell = (int32_t *)(ws + L.t_cell);
    float4 *t_pos = (float4 *)(ws + L.t_pos);
    float4 *t_vel = (float4 *)(ws + L.t_vel);
    uint32_t *t_info = (uint32_t *)(ws + L.t_info);
    float4 *pos = (float4 *)parts->pos;
    float4 *vel = (float4 *)parts->vel;

    const CellDims dims{grid->ncell[0], grid->ncell[1], grid->ncell[2], grid->periodic};
    const int nbk = n_cells + 1;

    const int cap_ids = brick_table_cap(cap);
    int32_t *table = neibs_brick ? brick_table(reinterpret_cast<int32_t *>(neibs_brick), cap, max_neibs) : nullptr;
    uint8_t *flags = neibs_brick ? (uint8_t *)(ws + L.flags) : nullptr;
    int32_t *active = (int32_t *)(ws + L.active);
    const int64_t flag_words = neibs_brick ? (n_cells + 3) / 4 : 0;
    const int64_t zero_items = nbk > flag_words ? nbk : flag_words;
    const unsigned fill_blocks = sph_blocks(zero_items, kThreads) < 4096u ? sph_blocks(zero_items, kThreads) : 4096u;
    k_build_zero<<<fill_blocks, kThreads, 0, s>>>(nbk, cnt, cursor, d_status, flag_words, (int32_t *)flags, active,
                                                  table, table ? table + cap_ids + 1 : nullptr);
    SPH_CHECK_LAUNCH();
    if (n > 0) {
        k_rebin_count<<<sph_blocks(n, kThreads), kThreads, 0, s>>>(
            n, parts->cell, pos, dims, grid->cell_size[0], grid->cell_size[1], grid->cell_size[2],
            grid->cell_base, n_cells, cnt);
        SPH_CHECK_LAUNCH();
    }
    const int np = (nbk + kScanTile - 1) / kScanTile;
    k_scan_reduce<<<np, kThreads, 0, s>>>(cnt, nbk, partials);
    k_scan_partials<<<1, kThreads, 0, s>>>(partials, np, start + nbk);
    k_scan_apply<<<np, kThreads, 0, s>>>(cnt, nbk, partials, start);
    SPH_CHECK_LAUNCH();
    k_cell_ranges<<<sph_blocks(n_cells, kThreads), kThreads, 0, s>>>(n_cells, start, cell_start, cell_end, n,
                                                                     d_status);
    SPH_CHECK_LAUNCH();
    if (n > 0) {
        k_scatter<<<sph_blocks(n, kThreads), kThreads, 0, s>>>(n, parts->cell, grid->cell_base, n_cells,
                                                                start, cursor, perm_a);
        k_cell_sort<<<sph_blocks((n + kWave - 1) / kWave, kThreads / kWave), kThreads, 0, s>>>(
            n, parts->cell, grid->cell_base, n_cells, start, perm_a, parts->info, perm_b);
        k_gather<<<sph_blocks(n, kThreads), kThreads, 0, s>>>(n, perm_b, parts->cell, pos, vel, parts->info,
                                                               t_cell, t_pos, t_vel, t_info, perm_out, d_status);
        SPH_CHECK_LAUNCH();
        const float rs2 = params->r_search * params->r_search;
        with_shape(shape, [&]<int BX, int BY, int BZ>() {
            const BrickGrid G = brick_grid<BX, BY, BZ>(grid->ncell, grid->periodic);
            const unsigned bricks = (unsigned)G.nbx * G.nby * G.nbz;
            constexpr int NT = brick_threads(BX * BY * BZ);
            // brick activity from the (exclusive-scan) cell starts: start[c + 1] is the end of cell c
            k_active_bricks<BX, BY, BZ><<<sph_blocks(bricks, 256), 256, 0, s>>>(start, start + 1, G, active, nullptr);
            k_build_brick<BX, BY, BZ, NT, kBuildCap><<<bricks, NT, 0, s>>>(
                n, max_neibs, t_pos, t_info, start, G, grid->cell_size[0], grid->cell_size[1], grid->cell_size[2],
                rs2, active, neibs, neibs_brick, neib_count, d_status);
        });
        k_copy_state<<<sph_blocks(n, kThreads), kThreads, 0, s>>>(n, t_cell, t_pos, t_vel, t_info, parts->cell,
                                                                   pos, vel, parts->info, neib_count,
                                                                   grid->cell_base, n_cells, flags);
        SPH_CHECK_LAUNCH();
    }
    if (neibs_brick) {
        // the table of bricks with a pair behind the brick-local lists, for
        // the derivative kernels (heavy bricks first: at least 12 particles
        // per inner cell), from the cell flags k_copy_state set
        with_shape(shape, [&]<int BX, int BY, int BZ>() {
            const BrickGrid G = brick_grid<BX, BY, BZ>(grid->ncell, grid->periodic);
            const unsigned bricks = (unsigned)G.nbx * G.nby * G.nbz;
            k_active_bricks<BX, BY, BZ><<<sph_blocks(bricks, 256), 256, 0, s>>>(
                start, start + 1, G, table, flags, table + cap_ids + 1, 12 * BX * BY * BZ, cap_ids);
        });
        SPH_CHECK_LAUNCH();
    }
    return SPH_OK;
}
