// Time derivatives of the WCSPH step ("forces"): continuity, Cole equation
// of state, golden-rule pressure gradient with Monaghan artificial viscosity
// and the optional Morris laminar term, Wendland C2 kernel (arXiv:2207.11328,
// eq. mass-cont-sph1, eq. ns-sph1, section "Minimizing complexity", listing
// l:ktemplate).
//
// Layout of the work on gfx950:
// * A prologue pass evaluates the equation of state once per particle
//   (P/rho^2 and alpha h c), so the pair loop gathers 8 bytes instead of
//   recomputing a 6th-order polynomial and a reciprocal per pair.
// * One lane per central particle; the list is neighbour-major inside tiles
//   of 64 particles, so slot k of a wave is one contiguous 256-byte row and
//   its address is one 32-bit offset from the lane's tile base.
// * The trip count is the wave's largest list (a scalar), lanes past their
//   own count are masked, and fluid and boundary segments are walked in one
//   loop (slot k < nf from the front, the rest from the back), so there is
//   no divergent control flow in the pair loop.
// * Loads are software-pipelined: list entries two pairs ahead, neighbour
//   data one pair ahead, so each wave keeps several gathers in flight.
#include <hip/hip_runtime.h>
#include <math.h>

#include "sph_device.h"

using namespace sph;

namespace {

constexpr int kThreads = 256;
// pairs in flight per lane in the derivative loop
#ifndef SPH_FORCES_DEPTH
#define SPH_FORCES_DEPTH 4
#endif
constexpr int kDepth = SPH_FORCES_DEPTH;

struct ForceConst {
    float csx, csy, csz;
    float rho0, inv_rho0, B, c0;
    float lim2;      // fl32(2h)^2: interaction iff r2 < lim2
    float inv_h;
    float fcoeff;    // 105 / (128 pi h^5)
    float alpha_h;   // alpha * h
    float eps_h2;    // eps * h^2
    float four_nu;   // 4 nu
    float diff;      // 2 delta h c0 (density diffusion)
    int max_neibs;
};

// Cole EOS for gamma = 7 in the expanded form P = B d (7 + 21d + 35d^2 +
// 35d^3 + 21d^4 + 7d^5 + d^6), d = (rho - rho0)/rho0 (exact expansion of
// (1 + d)^7 - 1, full relative accuracy near rho0).  aux = (P/rho^2,
// alpha h c / 2) with c = c0 (1 + d)^3.
// Also (brick form): zeroes the active-brick counter and the derivatives of
// particles the last build dropped (cell < 0), which no brick visits.
__global__ __launch_bounds__(kThreads) void k_eos(int n, const float4 *__restrict__ vel, float2 *__restrict__ aux,
                                                  const int32_t *__restrict__ cell,
                                                  const float *__restrict__ cell_alpha, int cell_base, float h,
                                                  ForceConst C, int32_t *__restrict__ active,
                                                  float4 *__restrict__ out)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (active && i == 0) active[0] = 0;
    if (i >= n) return;
    float alpha_h = C.alpha_h;
    if (cell_alpha || out) {
        const int c = cell[i];
        if (cell_alpha && c >= 0) alpha_h = cell_alpha[c - cell_base] * h;
        if (out && c < 0) out[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    const float rho = vel[i].w;
    const float d = (rho - C.rho0) * C.inv_rho0;
    float poly = 7.0f + d;
    poly = fmaf(poly, d, 21.0f);
    poly = fmaf(poly, d, 35.0f);
    poly = fmaf(poly, d, 35.0f);
    poly = fmaf(poly, d, 21.0f);
    poly = fmaf(poly, d, 7.0f);
    const float P = C.B * d * poly;
    const float inv_rho = 1.0f / rho;
    const float a = 1.0f + d;
    aux[i] = make_float2(P * inv_rho * inv_rho, 0.5f * alpha_h * (C.c0 * a * a * a));
}

// Cell difference k_d in {-1, 0, 1} of axis d, stored as a two's-complement
// 2-bit field at bit 26 + 2d of a list entry.
__device__ __forceinline__ float entry_k(uint32_t e, int axis)
{
    return (float)((int32_t)(e << (4 - 2 * axis)) >> 30);
}

__device__ __forceinline__ int list_slot(int k, int nf, int last, int M)
{
    const int kk = min(k, last);
    return kk < nf ? kk : M - 1 + nf - kk;
}

struct PairAcc {
    float ax, ay, az, dr;
};

// Model template parameter: bit 0 = Morris laminar viscosity, bit 1 =
// density diffusion between fluid particles.
constexpr int kLaminar = 1, kDiffusion = 2;

// One pair (i, j) of the derivative sums, branch-free; contributes only when
// `valid` (slot inside i's list) and r < 2h.  mfj = m_j times the Wendland
// coefficient 105/(128 pi h^5); ai.y, aj.y = alpha h c / 2 (so the mean of
// the sound speeds and the min(u.x, 0) of Monaghan's term come out of one
// sum and one subtraction: (ai.y + aj.y)(w - |w|) = alpha h (c_i + c_j) min(w, 0)).
// pair_fluid: both particles are fluid (density diffusion applies).
template <int VISC>
__device__ __forceinline__ void pair_core(PairAcc &A, float xx, float xy, float xz, const float4 &vi,
                                          const float2 &ai, float mfj, const float4 &vj, const float2 &aj,
                                          bool valid, bool pair_fluid, const ForceConst &C)
{
    const float r2 = fmaf(xx, xx, fmaf(xy, xy, xz * xz));
    const bool inter = valid && (r2 < C.lim2);
    const float r = __builtin_amdgcn_sqrtf(r2);
    const float qm2 = fmaf(r, C.inv_h, -2.0f);
    const float mF = (qm2 * qm2) * (qm2 * mfj);  // m_j F_ij
    const float ux = vi.x - vj.x;
    const float uy = vi.y - vj.y;
    const float uz = vi.z - vj.z;
    const float udx = fmaf(ux, xx, fmaf(uy, xy, uz * xz));
    A.dr = inter ? fmaf(mF, udx, A.dr) : A.dr;
    // Monaghan: Pi = -alpha h (c_i + c_j)/2 min(u.x, 0) / ((rho_i + rho_j)/2 (r^2 + eps h^2))
    const float den = (vi.w + vj.w) * (r2 + C.eps_h2);
    const float visc = -(ai.y + aj.y) * (udx - fabsf(udx)) * __builtin_amdgcn_rcpf(den);
    const float coef = inter ? -mF * (ai.x + aj.x + visc) : 0.0f;
    A.ax = fmaf(coef, xx, A.ax);
    A.ay = fmaf(coef, xy, A.ay);
    A.az = fmaf(coef, xz, A.az);
    if (VISC & kLaminar) {
        const float lam = inter ? C.four_nu * mF * __builtin_amdgcn_rcpf(vi.w + vj.w) : 0.0f;
        A.ax = fmaf(lam, ux, A.ax);
        A.ay = fmaf(lam, uy, A.ay);
        A.az = fmaf(lam, uz, A.az);
    }
    if (VISC & kDiffusion) {
        // Molteni-Colagrossi: 2 delta h c0 (rho_i - rho_j) m_j F r^2 / ((r^2 + eps h^2) rho_j)
        const float dd = C.diff * (vi.w - vj.w) * mF * r2 * __builtin_amdgcn_rcpf((r2 + C.eps_h2) * vj.w);
        A.dr = (inter && pair_fluid) ? A.dr + dd : A.dr;
    }
}

template <int VISC>
__device__ __forceinline__ void pair_terms(PairAcc &A, uint32_t e, const float4 &pi, const float4 &vi,
                                           const float2 &ai, const float4 &pj, const float4 &vj, const float2 &aj,
                                           bool valid, bool pair_fluid, const ForceConst &C)
{
    // separation, bit-identical to the list predicate: x = k cs + (o_i - o_j)
    const float xx = fmaf(entry_k(e, 0), C.csx, pi.x - pj.x);
    const float xy = fmaf(entry_k(e, 1), C.csy, pi.y - pj.y);
    const float xz = fmaf(entry_k(e, 2), C.csz, pi.z - pj.z);
    pair_core<VISC>(A, xx, xy, xz, vi, ai, pj.w * C.fcoeff, vj, aj, valid, pair_fluid, C);
}

// Pairs of one lane's list gathered from global memory, in list order.
// Software pipeline over a ring of D pair slots, unrolled by D: slot s holds
// the neighbour data of pair k + s (requested D pairs before it is used) and
// the list entry of pair k + s + D (requested 2 D pairs ahead).  Neighbour
// data registers are only ever written by loads, so the loop carries no copy
// of an in-flight value.
template <int VISC, int D>
__device__ __forceinline__ void gather_pairs(PairAcc &A, const uint32_t *tile, int nf, int nt, int ntw, int M,
                                             uint32_t jmax, const float4 *__restrict__ pos,
                                             const float4 *__restrict__ vel, const float2 *__restrict__ aux,
                                             const float4 &pi, const float4 &vi, const float2 &ai,
                                             bool central_fluid, const ForceConst &C)
{
    const int last = max(nt - 1, 0);
    uint32_t e[D], en[D];
    float4 P[D], V[D];
    float2 X[D];
#pragma unroll
    for (int s = 0; s < D; ++s) {
        e[s] = tile[list_slot(s, nf, last, M) * kWave];
        en[s] = tile[list_slot(s + D, nf, last, M) * kWave];
    }
#pragma unroll
    for (int s = 0; s < D; ++s) {
        const uint32_t j = min(e[s] & kIndexMask, jmax);
        P[s] = pos[j];
        V[s] = vel[j];
        X[s] = aux[j];
    }
    for (int k = 0; k < ntw; k += D) {
#pragma unroll
        for (int s = 0; s < D; ++s) {
            pair_terms<VISC>(A, e[s], pi, vi, ai, P[s], V[s], X[s], k + s < nt, central_fluid && k + s < nf, C);
            e[s] = en[s];
            const uint32_t j = min(e[s] & kIndexMask, jmax);
            P[s] = pos[j];
            V[s] = vel[j];
            X[s] = aux[j];
            en[s] = tile[list_slot(k + s + 2 * D, nf, last, M) * kWave];
        }
    }
}

template <int VISC>
__global__ __launch_bounds__(kThreads) void k_forces(int n, const float4 *__restrict__ pos,
                                                     const float4 *__restrict__ vel,
                                                     const float2 *__restrict__ aux,
                                                     const uint32_t *__restrict__ neibs,
                                                     const uint32_t *__restrict__ count,
                                                     const uint32_t *__restrict__ info,
                                                     float4 *__restrict__ out, ForceConst C)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    const int lane = threadIdx.x % kWave;
    const int ii = min(i, n - 1);  // lanes past the end load in bounds and store nothing
    const int M = C.max_neibs;
    const uint32_t cnt = i < n ? count[i] : 0u;
    // counts and indices are clamped: a stale or foreign list gives wrong
    // numbers but never an out-of-bounds access
    const int nf = min((int)(cnt & 0xFFFFu), M);
    const int nt = min(nf + (int)(cnt >> 16), M);
    const int ntw = __builtin_amdgcn_readfirstlane(wave_max(nt));
    if (ntw == 0) {
        if (i < n) out[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        return;
    }
    // a wave is exactly one 64-particle tile of the list (wave-uniform base)
    const int tile_id = __builtin_amdgcn_readfirstlane(i / kWave);
    const uint32_t *tile = neibs + (size_t)tile_id * (kWave * M);
    const uint32_t jmax = (uint32_t)(n - 1);

    const float4 pi = pos[ii];
    const float4 vi = vel[ii];
    const float2 ai = aux[ii];
    PairAcc A = {0.0f, 0.0f, 0.0f, 0.0f};

    const bool central_fluid = (VISC & kDiffusion) ? ptype(info[ii]) != kBoundary : true;
    gather_pairs<VISC, kDepth>(A, tile + lane, nf, nt, ntw, M, jmax, pos, vel, aux, pi, vi, ai, central_fluid, C);
    if (i < n) out[i] = nt > 0 ? make_float4(A.ax, A.ay, A.az, A.dr) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// ---------------------------------------------------------------------------
// Cell-brick variant of the derivative kernel (the cell perspective of section
// "Changing perspective: from the particle to the cell" applied to the
// derivatives).  A workgroup owns a brick of cells; it first copies
// the particles of the brick and of its one-cell halo (every possible
// neighbour of its particles) from HBM/L2 into LDS with coalesced loads, one
// contiguous cell range after another, then each lane walks the list of one
// central particle of the brick and reads the neighbour data from LDS.  The
// 64 lanes of a wave read neighbours scattered over dozens of cache lines,
// which the global-gather kernel pays in L1/L2 request throughput.
//
// The lists are the brick-local ones of the build: entry k is the
// neighbour's LDS slot itself (uint16, fluid then boundary contiguous), so a
// pair costs no index decoding.  Staged positions are relative to the centre
// cell of the brick, o + s cs with s in {-2, ..., 2} per axis, so the
// separation is one subtraction: its rounding error is a few ulp of 2.5 cs,
// not of cs (the list predicate, which must be exact, is not evaluated here;
// the r < 2h mask only differs from the exact one where the kernel weight is
// of order 1e-20).  A brick whose halo does not fit in LDS reads the global
// lists and the global state with the arithmetic of k_forces.

// Pairs of one lane's brick-local list, read from LDS.  The list arrives in
// 16-byte groups of 8 entries (one load per 8 pairs), requested two groups
// ahead; the staged data of pair k + R is requested while pair k is computed
// (a ring of R slots, R dividing 8 so the ring phase is the same in every
// group).
#ifndef SPH_BRICK_RING
#define SPH_BRICK_RING 2
#endif
constexpr int kRing = SPH_BRICK_RING;
static_assert(kBrickGroup % kRing == 0, "ring must divide the group");

__device__ __forceinline__ uint32_t group_entry(const uint4 &g, int s)
{
    const uint32_t w = (s >> 1) == 0 ? g.x : (s >> 1) == 1 ? g.y : (s >> 1) == 2 ? g.z : g.w;
    return (s & 1) ? (w >> 16) : (w & 0xFFFFu);
}

template <int VISC, int NT>
__device__ __forceinline__ void brick_pairs_lds(PairAcc &A, const uint4 *lg, int nt, int ntw, int total,
                                                const float4 *__restrict__ sP, const float4 *__restrict__ sV,
                                                const float2 *__restrict__ sA, const float4 &pi, const float4 &vi,
                                                const float2 &ai, const ForceConst &C)
{
    constexpr int GS = kWave;  // uint4 stride between groups of one lane
    const int lastg = max(nt - 1, 0) / kBrickGroup;
    const uint32_t smax = (uint32_t)(total - 1);
    float4 P[kRing], V[kRing];
    float2 X[kRing];
    auto fetch = [&](uint32_t slot, float4 &p, float4 &v, float2 &x) {
        const uint32_t sl = min(slot, smax);  // a stale list stays inside the staged range
        p = sP[sl];
        v = sV[sl];
        x = sA[sl];
    };
    uint4 gc = lg[0];
    uint4 gn = lg[min(1, lastg) * GS];
#pragma unroll
    for (int r = 0; r < kRing; ++r) fetch(group_entry(gc, r), P[r], V[r], X[r]);
    for (int k = 0; k < ntw; k += kBrickGroup) {
        const uint4 gnn = lg[min(k / kBrickGroup + 2, lastg) * GS];
#pragma unroll
        for (int s = 0; s < kBrickGroup; ++s) {
            const int r = s % kRing;
            // staged w = +-(m_j x Wendland coefficient), negative for boundary particles
            pair_core<VISC>(A, pi.x - P[r].x, pi.y - P[r].y, pi.z - P[r].z, vi, ai, fabsf(P[r].w), V[r], X[r],
                            k + s < nt, pi.w > 0.0f && P[r].w > 0.0f, C);
            const int s2 = s + kRing;
            fetch(s2 < kBrickGroup ? group_entry(gc, s2) : group_entry(gn, s2 - kBrickGroup), P[r], V[r], X[r]);
        }
        gc = gn;
        gn = gnn;
    }
}

template <int VISC, int BX, int BY, int BZ, int NT, int CAP>
__global__ __launch_bounds__(NT) void k_forces_brick(int n, const float4 *__restrict__ pos,
                                                     const float4 *__restrict__ vel,
                                                     const float2 *__restrict__ aux,
                                                     const uint32_t *__restrict__ neibs,
                                                     const uint16_t *__restrict__ neibs_brick,
                                                     const uint32_t *__restrict__ count,
                                                     const int32_t *__restrict__ cell_start,
                                                     const int32_t *__restrict__ cell_end,
                                                     const int32_t *__restrict__ active,
                                                     const uint32_t *__restrict__ info,
                                                     float4 *__restrict__ out, ForceConst C, BrickGrid G)
{
    using St = Staging<BX, BY, BZ>;
    constexpr int SX = BX + 2, SY = BY + 2, SZ = BZ + 2;
    constexpr int S = SX * SY * SZ;  // staged cells
    constexpr int NI = BX * BY * BZ; // inner cells
    static_assert(S <= NT && NI <= NT, "one thread per cell");
    __shared__ float4 sP[CAP];  // brick-relative offset, mass x Wendland coefficient
    __shared__ float4 sV[CAP];
    __shared__ float2 sA[CAP];
    __shared__ int cBase[S + 1];
    __shared__ int cDelta[S];
    __shared__ int iBase[NI + 1];
    __shared__ int iStart[NI];
    __shared__ int wsum[NT / kWave];

    const int tid = threadIdx.x;
    // active[0] = number of bricks holding particles, active[1 + k] = brick id
    if ((int)blockIdx.x >= active[0]) return;
    const int b = active[1 + blockIdx.x];
    const int cx0 = (b % G.nbx) * BX, cy0 = ((b / G.nbx) % G.nby) * BY, cz0 = (b / (G.nbx * G.nby)) * BZ;

    // 1. ranges of the staged cells and their LDS bases (the staging order of
    //    the list build)
    int st = 0, cnt = 0;
    if (tid < S) {
        int gx = cx0 - 1 + St::sx_of(tid), gy = cy0 - 1 + St::sy_of(tid), gz = cz0 - 1 + St::sz_of(tid);
        const bool ok = wrap_axis(gx, G.nx, G.periodic & 1u) && wrap_axis(gy, G.ny, (G.periodic >> 1) & 1u) &&
                        wrap_axis(gz, G.nz, (G.periodic >> 2) & 1u);
        if (ok) {
            const int lin = gx + G.nx * (gy + G.ny * gz);
            st = cell_start[lin];
            cnt = cell_end[lin] - st;
        }
    }
    int total;
    const int ex = block_scan<NT>(cnt, total, wsum);
    if (tid < S) {
        cBase[tid] = ex;
        cDelta[tid] = ex - st;
    }
    if (tid == 0) cBase[S] = total;
    __syncthreads();
    // inner cells (x fastest: each inner row is one contiguous particle range)
    int icnt = 0, ist = 0;
    // inner cells past the grid edge hold no centrals (on a periodic axis the
    // staged copy would be the wrapped cell, owned by another brick)
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
    __syncthreads();
    const bool use_lds = total <= CAP;
    // central particle of lane q (binary search over the inner cells)
    auto central = [&](int q, int &u, int &i) {
        int lo = 0, hi = NI - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (iBase[mid] <= q) lo = mid;
            else hi = mid - 1;
        }
        u = lo;
        i = iStart[u] + (q - iBase[u]);
    };
    // the list count of the first pass is requested before the staging loads
    // so the two latencies overlap
    int u0, i0;
    central(min(tid, nc - 1), u0, i0);
    const uint32_t cnt0 = tid < nc ? count[i0] : 0u;
    if (use_lds) {
        // 2. stage the brick and its halo: one wave per row of SX staged
        //    cells (x-consecutive, so one contiguous LDS range and, away from
        //    a periodic seam, one contiguous global range), lanes over the
        //    row's particles
        const int wave = tid / kWave, lane = tid % kWave;
        for (int r = wave; r < SY * SZ; r += NT / kWave) {
            const int t0 = r * SX;
            const int b0 = cBase[t0], b1 = cBase[t0 + SX];
            int e[SX - 1];
#pragma unroll
            for (int c = 0; c < SX - 1; ++c) e[c] = cBase[t0 + 1 + c];
            const float sy = (float)(r / SZ - 2), sz = (float)(r % SZ - 2);
            for (int s2 = b0 + lane; s2 < b1; s2 += kWave) {
                int c = 0;
#pragma unroll
                for (int k = 0; k < SX - 1; ++k) c += s2 >= e[k] ? 1 : 0;
                const int j = s2 - cDelta[t0 + c];
                const float4 p = pos[j];
                const float sx = (float)(c - 2);
                // w = m x Wendland coefficient, negated for boundary particles
                // when the density diffusion needs the type
                const float mf = p.w * C.fcoeff;
                sP[s2] = make_float4(fmaf(sx, C.csx, p.x), fmaf(sy, C.csy, p.y), fmaf(sz, C.csz, p.z),
                                     ((VISC & kDiffusion) && ptype(info[j]) == kBoundary) ? -mf : mf);
                sV[s2] = vel[j];
                sA[s2] = aux[j];
            }
        }
    }
    __syncthreads();

    // 3. one lane per central particle of the brick
    const int M = C.max_neibs;
    const uint32_t jmax = (uint32_t)(n - 1);
    for (int q0 = 0; q0 < nc; q0 += NT) {
        const int q = q0 + tid;
        const bool act = q < nc;
        int u = u0, i = i0;
        uint32_t cntw = cnt0;
        if (q0 > 0) {
            central(act ? q : nc - 1, u, i);
            cntw = act ? count[i] : 0u;
        }
        const int nf = min((int)(cntw & 0xFFFFu), M);
        const int nt = min(nf + (int)(cntw >> 16), M);
        const int ntw = __builtin_amdgcn_readfirstlane(wave_max(nt));
        PairAcc A = {0.0f, 0.0f, 0.0f, 0.0f};
        if (ntw > 0) {
            const size_t toff = (size_t)(i / kWave) * (kWave * M) + (i % kWave);
            if (use_lds) {
                const int tc = St::inner(u);
                const int si = i + cDelta[tc];
                const uint4 *lg = (const uint4 *)(neibs_brick + brick_entry(i, 0, brick_groups(M)));
                brick_pairs_lds<VISC, NT>(A, lg, nt, ntw, total, sP, sV, sA, sP[si], sV[si], sA[si], C);
            } else {
                // (a shallow pipeline: this path shares the register budget of
                // the LDS path and runs only where a halo overflows)
                const bool central_fluid = (VISC & kDiffusion) ? ptype(info[i]) != kBoundary : true;
                gather_pairs<VISC, 2>(A, neibs + toff, nf, nt, ntw, M, jmax, pos, vel, aux, pos[i], vel[i], aux[i],
                                      central_fluid, C);
            }
        }
        if (act) out[i] = nt > 0 ? make_float4(A.ax, A.ay, A.az, A.dr) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
}

__global__ __launch_bounds__(kThreads) void k_count_interactions(int n, const float4 *__restrict__ pos,
                                                                 const uint32_t *__restrict__ neibs,
                                                                 const uint32_t *__restrict__ count,
                                                                 ForceConst C,
                                                                 unsigned long long *__restrict__ total)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    unsigned long long c = 0;
    if (i < n) {
        const int M = C.max_neibs;
        const uint32_t cnt = count[i];
        const int nf = min((int)(cnt & 0xFFFFu), M);
        const int nt = min(nf + (int)(cnt >> 16), M);
        const uint32_t jmax = (uint32_t)(n - 1);
        const uint32_t *tile = neibs + (size_t)(i / kWave) * (kWave * M) + (i % kWave);
        const float4 pi = pos[i];
        for (int k = 0; k < nt; ++k) {
            const uint32_t e = tile[list_slot(k, nf, nt - 1, M) * kWave];
            const float4 pj = pos[min(e & kIndexMask, jmax)];
            const float r2 = predicate_r2(pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, entry_k(e, 0) * C.csx,
                                          entry_k(e, 1) * C.csy, entry_k(e, 2) * C.csz);
            c += r2 < C.lim2 ? 1ull : 0ull;
        }
    }
    c = wave_sum(c);
    if ((threadIdx.x % kWave) == 0 && c) atomicAdd(total, c);
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

bool make_const(const sph_grid *g, const sph_params *p, int max_neibs, ForceConst &C)
{
    if (!(p->h > 0.0f) || !(p->rho0 > 0.0f) || !(p->c0 > 0.0f) || p->gamma != 7.0f) return false;
    if (p->visc_model != 0 && p->visc_model != 1) return false;
    if (!(p->delta >= 0.0f) || !(p->delta < 1e30f)) return false;
    for (int d = 0; d < 3; ++d)
        if (!(g->cell_size[d] > 0.0f)) return false;
    C.csx = g->cell_size[0];
    C.csy = g->cell_size[1];
    C.csz = g->cell_size[2];
    C.rho0 = p->rho0;
    C.inv_rho0 = (float)(1.0 / (double)p->rho0);
    C.B = (float)((double)p->rho0 * (double)p->c0 * (double)p->c0 / (double)p->gamma);
    C.c0 = p->c0;
    const float two_h = 2.0f * p->h;
    C.lim2 = two_h * two_h;
    C.inv_h = (float)(1.0 / (double)p->h);
    const double h = p->h;
    C.fcoeff = (float)(105.0 / (128.0 * M_PI * h * h * h * h * h));
    C.alpha_h = (float)((double)p->alpha * h);
    C.eps_h2 = (float)((double)p->eps_visc * h * h);
    C.four_nu = (float)(4.0 * (double)p->nu);
    C.diff = (float)(2.0 * (double)p->delta * h * (double)p->c0);
    C.max_neibs = max_neibs;
    return true;
}

bool common_args(const sph_grid *g, const sph_params *p, const sph_particles *parts, const uint32_t *neibs,
                 const uint32_t *count, int max_neibs)
{
    if (!g || !p || !parts) return false;
    if (parts->n < 0 || parts->capacity < parts->n || parts->capacity > SPH_MAX_CAPACITY) return false;
    if (parts->n > 0 && (!parts->pos || !parts->vel || !neibs || !count)) return false;
    if (max_neibs < 1 || max_neibs > 65535) return false;
    return true;
}

size_t aux_bytes(int64_t capacity) { return (size_t)((sizeof(float2) * capacity + 255) & ~(int64_t)255); }

}  // namespace

extern "C" size_t sph_forces_workspace_bytes(int32_t capacity, int32_t n_cells)
{
    if (capacity < 0 || n_cells < 0) return 0;
    // per-particle EOS terms, then the active-brick list (at most one brick per cell)
    return aux_bytes(capacity > 0 ? capacity : 1) + sizeof(int32_t) * ((size_t)n_cells + 1) + 256;
}

// LDS capacity (staged particles, 40 bytes each) per brick shape: the halo
// of a brick at the h = 1.3 dp, r_s = 2.86 dp lattice density holds up to
// about 27 particles per staged cell (3 x 4 x 3: 150 cells, 3825 at most in
// the 1.62M dam break; 3 x 3 x 3: 125 cells, 3375; 3 x 2 x 3: 100 cells).
// Measured on the 1.62M dam break (one workgroup per CU in every case):
// 3 x 4 x 3 277 us, 3 x 3 x 3 357 us, 4 x 3 x 3 425 us (1% of its bricks
// overflow the LDS there).
constexpr int brick_cap(int BX, int BY, int BZ) { return BX * BY * BZ >= 36 ? 4000 : (BX * BY * BZ >= 27 ? 3400 : 2750); }

template <int VISC>
void launch_brick(const sph_grid *grid, int shape, int n, const float4 *pos, const float4 *vel, const float2 *aux,
                  const uint32_t *neibs, const uint16_t *neibs_brick, const uint32_t *count,
                  const int32_t *cell_start, const int32_t *cell_end, int32_t *active, const uint32_t *info,
                  float4 *out, const ForceConst &C, hipStream_t s)
{
    with_shape(shape, [&]<int BX, int BY, int BZ>() {
        const BrickGrid G = brick_grid<BX, BY, BZ>(grid->ncell, grid->periodic);
        const unsigned blocks = (unsigned)G.nbx * G.nby * G.nbz;
        constexpr int NT = brick_threads(BX * BY * BZ);
        // (active[0] was zeroed by k_eos)
        k_active_bricks<BX, BY, BZ><<<sph_blocks(blocks, 256), 256, 0, s>>>(cell_start, cell_end, G, active);
        k_forces_brick<VISC, BX, BY, BZ, NT, brick_cap(BX, BY, BZ)><<<blocks, NT, 0, s>>>(
            n, pos, vel, aux, neibs, neibs_brick, count, cell_start, cell_end, active, info, out, C, G);
    });
}

extern "C" sph_status sph_forces(const sph_grid *grid, const sph_params *params, const sph_particles *parts,
                                 const uint32_t *neibs, const uint32_t *neib_count, int32_t max_neibs,
                                 const int32_t *cell_start, const int32_t *cell_end,
                                 const uint16_t *neibs_brick, float *forces, void *workspace,
                                 size_t workspace_bytes, void *stream)
{
    if (!common_args(grid, params, parts, neibs, neib_count, max_neibs)) return SPH_ERR_ARG;
    if (parts->n > 0 && !forces) return SPH_ERR_ARG;
    ForceConst C;
    if (!make_const(grid, params, max_neibs, C)) return SPH_ERR_ARG;
    const int shape = brick_shape_index(grid->brick);
    if (shape < 0) return SPH_ERR_ARG;
    const int64_t n_cells = (int64_t)grid->ncell[0] * grid->ncell[1] * grid->ncell[2];
    if (n_cells <= 0 || n_cells > INT32_MAX - 1) return SPH_ERR_ARG;
    if (!workspace || workspace_bytes < sph_forces_workspace_bytes(parts->capacity, (int32_t)n_cells))
        return SPH_ERR_WORKSPACE;
    const int n = parts->n;
    if (n == 0) return SPH_OK;
    hipStream_t s = (hipStream_t)stream;
    const float4 *pos = (const float4 *)parts->pos;
    const float4 *vel = (const float4 *)parts->vel;
    float2 *aux = (float2 *)workspace;
    int32_t *active = (int32_t *)((char *)workspace + aux_bytes(parts->capacity > 0 ? parts->capacity : 1));
    float4 *out = (float4 *)forces;
    if (grid->cell_alpha && !parts->cell) return SPH_ERR_ARG;
    const bool bricks = cell_start && cell_end && neibs_brick;
    if (bricks && !parts->cell) return SPH_ERR_ARG;
    k_eos<<<sph_blocks(n, kThreads), kThreads, 0, s>>>(n, vel, aux, parts->cell, grid->cell_alpha, grid->cell_base,
                                                       params->h, C, bricks ? active : nullptr,
                                                       bricks ? out : nullptr);
    if ((params->delta != 0.0f) && !parts->info) return SPH_ERR_ARG;
    const int model = params->visc_model | (params->delta != 0.0f ? kDiffusion : 0);
    const uint32_t *info = parts->info;
    if (bricks) {
        // cell ranges and brick-local lists of the last build: LDS cell-brick
        // kernel (it writes the derivatives of every particle that lies in a
        // cell; particles dropped by the build were zeroed by k_eos)
        switch (model) {
        case 0: launch_brick<0>(grid, shape, n, pos, vel, aux, neibs, neibs_brick, neib_count, cell_start, cell_end,
                                active, info, out, C, s); break;
        case 1: launch_brick<1>(grid, shape, n, pos, vel, aux, neibs, neibs_brick, neib_count, cell_start, cell_end,
                                active, info, out, C, s); break;
        case 2: launch_brick<2>(grid, shape, n, pos, vel, aux, neibs, neibs_brick, neib_count, cell_start, cell_end,
                                active, info, out, C, s); break;
        default: launch_brick<3>(grid, shape, n, pos, vel, aux, neibs, neibs_brick, neib_count, cell_start,
                                 cell_end, active, info, out, C, s); break;
        }
    } else {
        const unsigned b = sph_blocks(n, kThreads);
        switch (model) {
        case 0: k_forces<0><<<b, kThreads, 0, s>>>(n, pos, vel, aux, neibs, neib_count, info, out, C); break;
        case 1: k_forces<1><<<b, kThreads, 0, s>>>(n, pos, vel, aux, neibs, neib_count, info, out, C); break;
        case 2: k_forces<2><<<b, kThreads, 0, s>>>(n, pos, vel, aux, neibs, neib_count, info, out, C); break;
        default: k_forces<3><<<b, kThreads, 0, s>>>(n, pos, vel, aux, neibs, neib_count, info, out, C); break;
        }
    }
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

extern "C" sph_status sph_count_interactions(const sph_grid *grid, const sph_params *params,
                                             const sph_particles *parts, const uint32_t *neibs,
                                             const uint32_t *neib_count, int32_t max_neibs,
                                             unsigned long long *d_count, void *stream)
{
    if (!common_args(grid, params, parts, neibs, neib_count, max_neibs) || !d_count) return SPH_ERR_ARG;
    ForceConst C;
    if (!make_const(grid, params, max_neibs, C)) return SPH_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    k_zero_u64<<<1, 1, 0, s>>>(d_count);
    SPH_CHECK_LAUNCH();
    const int n = parts->n;
    if (n == 0) return SPH_OK;
    k_count_interactions<<<sph_blocks(n, kThreads), kThreads, 0, s>>>(n, (const float4 *)parts->pos, neibs,
                                                                      neib_count, C, d_count);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}
