// Pair loops of the time derivatives ("forces"): continuity, pressure
// gradient, artificial and laminar viscosity, density diffusion, for the
// smoothing kernel SPH_KERNEL_KIND (arXiv:2207.11328, eq. mass-cont-sph1,
// eq. ns-sph1, eq. mass-cont-sph2, eq. ns-sph2, section "Minimizing
// complexity", listing l:ktemplate).  This file is compiled once per kernel;
// each object holds every formulation / laminar term / diffusion instance of
// its kernel, in both kernel forms (global gather and LDS brick).
//
// Layout of the work on gfx950:
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

#include "forces_common.h"

#ifndef SPH_KERNEL_KIND
#error "compile with SPH_KERNEL_KIND set to one of the SPH_KERNEL_* values"
#endif

using namespace sph;

namespace {

constexpr int kThreads = 256;
// pairs in flight per lane in the derivative loop
#ifndef SPH_FORCES_DEPTH
#define SPH_FORCES_DEPTH 4
#endif
constexpr int kDepth = SPH_FORCES_DEPTH;

struct PairAcc {
    float ax, ay, az, dr;
};

// One pair (i, j) of the derivative sums, branch-free; contributes only when
// `valid` (slot inside i's list) and r < 2h.  mcj = m_j times the kernel
// coefficient c of F = c f(q); ai.y, aj.y = alpha h c / 2 (so the mean of
// the sound speeds and the min(u.x, 0) of Monaghan's term come out of one
// sum and one subtraction: (ai.y + aj.y)(w - |w|) = alpha h (c_i + c_j) min(w, 0));
// ai.x, aj.x = P/rho^2 (golden rule) or P (Landrini-Morris).
// pair_fluid: both particles are fluid (density diffusion applies).
// LDS: the form of the LDS brick loop, where a pair outside the support or
// past the list has m_j F set to zero and every term is computed (no branch,
// fewer registers); the global-gather loop keeps per-term selects, which the
// compiler turns into a branch that skips the term arithmetic and keeps more
// gathers in flight.  Both give the same values (the zeroed terms add +-0).
template <int MODEL, bool LDS>
__device__ __forceinline__ void pair_core(PairAcc &A, float xx, float xy, float xz, const float4 &vi,
                                          const float2 &ai, float mcj, const float4 &vj, const float2 &aj,
                                          bool valid, bool pair_fluid, const ForceConst &C)
{
    constexpr int KER = model_kernel(MODEL);
    const float r2 = fmaf(xx, xx, fmaf(xy, xy, xz * xz));
    bool inter = valid && (r2 < C.lim2);
    if constexpr (KER == SPH_KERNEL_QUADRATIC) inter = inter && r2 > 0.0f;  // its F is unbounded at r = 0
    const float r = __builtin_amdgcn_sqrtf(r2);
    // m_j F_ij; in the LDS form zero for a pair outside the support or past
    // the list (every term below is a finite factor times mF)
    const float mF0 = kernel_mF<KER>(mcj, r, r2, C.inv_h, C.inv_h2);
    const float mF = LDS ? (inter ? mF0 : 0.0f) : mF0;
    const float ux = vi.x - vj.x;
    const float uy = vi.y - vj.y;
    const float uz = vi.z - vj.z;
    const float udx = fmaf(ux, xx, fmaf(uy, xy, uz * xz));
    float pres;
    if constexpr (MODEL & kLandrini) {
        // (P_i + P_j)/(rho_i rho_j) and the continuity weight rho_i/rho_j
        const float inv_rj = __builtin_amdgcn_rcpf(vj.w);
        pres = (ai.x + aj.x) * (inv_rj * __builtin_amdgcn_rcpf(vi.w));
        A.dr = (LDS || inter) ? fmaf(mF * (vi.w * inv_rj), udx, A.dr) : A.dr;
    } else {
        pres = ai.x + aj.x;
        A.dr = (LDS || inter) ? fmaf(mF, udx, A.dr) : A.dr;
    }
    // Monaghan: Pi = -alpha h (c_i + c_j)/2 min(u.x, 0) / ((rho_i + rho_j)/2 (r^2 + eps h^2))
    const float d2 = r2 + C.eps_h2;
    const float den = (vi.w + vj.w) * d2;
    float vnum = -(ai.y + aj.y) * (udx - fabsf(udx));
    // laminar K form: + 4 K nu m_j F (u.x) / ((rho_i + rho_j)(r^2 + eps h^2)) x, the same denominator
    if constexpr (model_visc(MODEL) == kMonaghanK) vnum = fmaf(-C.k_four_nu, udx, vnum);
    const float inv_den = __builtin_amdgcn_rcpf(den);
    const float visc = vnum * inv_den;
    const float coef = (LDS || inter) ? -mF * (pres + visc) : 0.0f;
    A.ax = fmaf(coef, xx, A.ax);
    A.ay = fmaf(coef, xy, A.ay);
    A.az = fmaf(coef, xz, A.az);
    if constexpr (model_visc(MODEL) == kMorris) {
        // 1/(rho_i + rho_j) = (r^2 + eps h^2)/den: no second reciprocal
        const float lam = (LDS || inter) ? C.four_nu * mF * (d2 * inv_den) : 0.0f;
        A.ax = fmaf(lam, ux, A.ax);
        A.ay = fmaf(lam, uy, A.ay);
        A.az = fmaf(lam, uz, A.az);
    }
    if constexpr (MODEL & kDiffusion) {
        // Molteni-Colagrossi: 2 delta h c0 (rho_i - rho_j) m_j F r^2 / ((r^2 + eps h^2) rho_j)
        const float dd = C.diff * (vi.w - vj.w) * mF * r2 * __builtin_amdgcn_rcpf((r2 + C.eps_h2) * vj.w);
        A.dr = ((LDS || inter) && pair_fluid) ? A.dr + dd : A.dr;
    }
}

template <int MODEL>
__device__ __forceinline__ void pair_terms(PairAcc &A, uint32_t e, const float4 &pi, const float4 &vi,
                                           const float2 &ai, const float4 &pj, const float4 &vj, const float2 &aj,
                                           bool valid, bool pair_fluid, const ForceConst &C)
{
    // separation x = k cs + (o_i - o_j), each component bit-identical to the
    // list predicate's; r^2 is then formed with fused multiply-adds, so the
    // r < 2h decision can differ from an exactly rounded one by a rounding
    // of r^2
    const float xx = fmaf(entry_k(e, 0), C.csx, pi.x - pj.x);
    const float xy = fmaf(entry_k(e, 1), C.csy, pi.y - pj.y);
    const float xz = fmaf(entry_k(e, 2), C.csz, pi.z - pj.z);
    pair_core<MODEL, false>(A, xx, xy, xz, vi, ai, pj.w * C.fcoeff, vj, aj, valid, pair_fluid, C);
}

// Pairs of one lane's list gathered from global memory, in list order.
// Software pipeline over a ring of D pair slots, unrolled by D: slot s holds
// the neighbour data of pair k + s (requested D pairs before it is used) and
// the list entry of pair k + s + D (requested 2 D pairs ahead).  Neighbour
// data registers are only ever written by loads, so the loop carries no copy
// of an in-flight value.
// aux == nullptr: the neighbours' equation-of-state terms are evaluated from
// their densities (eos_terms, bit-identical to the gather form's prologue).
template <int MODEL, int D>
__device__ __forceinline__ void gather_pairs(PairAcc &A, const uint32_t *tile, int nf, int nt, int ntw, int M,
                                             uint32_t jmax, const float4 *__restrict__ pos,
                                             const float4 *__restrict__ vel, const float2 *__restrict__ aux,
                                             const int32_t *__restrict__ cell, const float4 &pi, const float4 &vi,
                                             const float2 &ai, bool central_fluid, const ForceConst &C)
{
    const int last = max(nt - 1, 0);
    uint32_t e[D], en[D];
    float4 P[D], V[D];
    float2 X[D];
    auto terms = [&](uint32_t j, const float4 &v) {
        return aux ? aux[j] : eos_terms(v.w, alpha_h_of((int)j, cell, C), C);
    };
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
        X[s] = terms(j, V[s]);
    }
    for (int k = 0; k < ntw; k += D) {
#pragma unroll
        for (int s = 0; s < D; ++s) {
            pair_terms<MODEL>(A, e[s], pi, vi, ai, P[s], V[s], X[s], k + s < nt, central_fluid && k + s < nf, C);
            e[s] = en[s];
            const uint32_t j = min(e[s] & kIndexMask, jmax);
            P[s] = pos[j];
            V[s] = vel[j];
            X[s] = terms(j, V[s]);
            en[s] = tile[list_slot(k + s + 2 * D, nf, last, M) * kWave];
        }
    }
}

template <int MODEL>
__global__ __launch_bounds__(kThreads) void k_forces(int n, const float4 *__restrict__ pos,
                                                     const float4 *__restrict__ vel,
                                                     const float2 *__restrict__ aux,
                                                     const uint32_t *__restrict__ neibs,
                                                     const uint32_t *__restrict__ count,
                                                     const uint32_t *__restrict__ info,
                                                     float4 *__restrict__ out, ForceConst C, Corrector K)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    const float tau = K.d_dt && !K.cell_scene ? (float)*K.d_dt : 0.0f;  // (the corrector's step)
    corrector_clock(K);
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
        if (i < n) {
            const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (out) out[i] = z;
            if (K.d_dt && K.cell[i] >= 0) corrector_at(i, z, vel[i], tau, K);
        }
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

    const bool central_fluid = (MODEL & kDiffusion) ? ptype(info[ii]) != kBoundary : true;
    gather_pairs<MODEL, kDepth>(A, tile + lane, nf, nt, ntw, M, jmax, pos, vel, aux, nullptr, pi, vi, ai,
                                central_fluid, C);
    if (i < n) {
        const float4 f = nt > 0 ? make_float4(A.ax, A.ay, A.az, A.dr) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (out) out[i] = f;
        if (K.d_dt && K.cell[i] >= 0) corrector_at(i, f, vi, tau, K);
    }
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
// not of cs (the list predicate, which must be exact, is not evaluated here).
// The r < 2h mask may therefore differ from an exactly rounded one for a
// pair within that error of the support edge: for the Wendland, cubic-spline
// and quadratic kernels such a pair weighs ~(q - 2)^2 or less, i.e. nothing
// in float32; the truncated Gaussian's F does not vanish at r = 2h, so there
// such a pair carries a finite weight and is counted by one side and not
// the other.  A brick whose halo does not fit in LDS reads the global
// lists and the global state with the arithmetic of k_forces.

// Pairs of one central's brick-local list, read from LDS, shared by two
// lanes: lane h of the pair takes the groups of 8 entries h, h + 2, h + 4, ...
// The list arrives in 16-byte groups (one load per 8 pairs), requested two
// iterations ahead; the staged data of pair k + R is requested while pair k
// is computed (a ring of R slots, R dividing 8 so the ring phase is the same
// in every group).
#ifndef SPH_BRICK_RING
#define SPH_BRICK_RING 2
#endif
constexpr int kRing = SPH_BRICK_RING;
static_assert(kBrickGroup % kRing == 0, "ring must divide the group");

template <int MODEL, int NT>
__device__ __forceinline__ void brick_pairs_lds(PairAcc &A, const uint4 *lg, int h, int nt, int ntw, int total,
                                                const float4 *__restrict__ sP, const float4 *__restrict__ sV,
                                                const float2 *__restrict__ sA, const float4 &pi, const float4 &vi,
                                                const float2 &ai, const ForceConst &C)
{
    constexpr int GS = kWave;  // uint4 stride between groups of one central
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
    uint4 gc = lg[min(h, lastg) * GS];
    uint4 gn = lg[min(h + 2, lastg) * GS];
#pragma unroll
    for (int r = 0; r < kRing; ++r) fetch(group_entry(gc, r), P[r], V[r], X[r]);
    for (int k = 0; k < ntw; k += 2 * kBrickGroup) {
        const int g0 = k / kBrickGroup + h;  // this lane's group
        const uint4 gnn = lg[min(g0 + 4, lastg) * GS];
        const int rem = nt - g0 * kBrickGroup;  // entries of the list from this group on
#pragma unroll
        for (int s = 0; s < kBrickGroup; ++s) {
            const int r = s % kRing;
            // staged w = +-(m_j x kernel coefficient), negative for boundary particles
            pair_core<MODEL, true>(A, pi.x - P[r].x, pi.y - P[r].y, pi.z - P[r].z, vi, ai, fabsf(P[r].w), V[r], X[r],
                            s < rem, pi.w > 0.0f && P[r].w > 0.0f, C);
            const int s2 = s + kRing;
            fetch(s2 < kBrickGroup ? group_entry(gc, s2) : group_entry(gn, s2 - kBrickGroup), P[r], V[r], X[r]);
        }
        gc = gn;
        gn = gnn;
    }
}

template <int MODEL, int BX, int BY, int BZ, int NT, int CAP>
__global__ __launch_bounds__(NT) void k_forces_brick(int n, const float4 *__restrict__ pos,
                                                     const float4 *__restrict__ vel,
                                                     const int32_t *__restrict__ cell,
                                                     const uint32_t *__restrict__ neibs,
                                                     const uint16_t *__restrict__ neibs_brick,
                                                     const uint32_t *__restrict__ count,
                                                     const int32_t *__restrict__ cell_start,
                                                     const int32_t *__restrict__ cell_end,
                                                     const int32_t *__restrict__ table, int cap_ids,
                                                     int32_t *__restrict__ next,
                                                     const uint32_t *__restrict__ info,
                                                     float4 *__restrict__ out, ForceConst C, BrickGrid G,
                                                     Corrector K)
{
    using St = Staging<BX, BY, BZ>;
    constexpr int SX = BX + 2, SY = BY + 2, SZ = BZ + 2;
    constexpr int S = SX * SY * SZ;  // staged cells
    constexpr int NI = BX * BY * BZ; // inner cells
    static_assert(S <= NT && NI <= NT, "one thread per cell");
    __shared__ float4 sP[CAP];  // brick-relative offset, mass x kernel coefficient
    __shared__ float4 sV[CAP];
    __shared__ float2 sA[CAP];
    // cell scans of the brick (two buffers: the next brick's are computed
    // ahead into the other one, see below)
    __shared__ int cBaseB[2][S + 1];
    __shared__ int cDeltaB[2][S];
    __shared__ int iBaseB[2][NI + 1];
    __shared__ int iStartB[2][NI];
    __shared__ int wsum[NT / kWave];
    __shared__ int sNext;
    __shared__ int sGroup;  // groups of centrals claimed in the brick, past the first NT / kWave
    __shared__ int sPre[4]; // scan ahead: claimed, next brick's list index, total, centrals
    // (corrector with a step per scene) each inner cell's scene (-1: none) and step
    __shared__ int sSc[NI];
    __shared__ float sTau[NI];
    static_assert(NI <= kWave, "one lane per inner cell in the scan ahead");

    // One resident workgroup per CU takes the bricks with a pair one at a time
    // from the counter `next`, heavy ones first (brick_at order; the build's
    // table): no workgroup is launched for an empty brick, the bricks'
    // different costs even out across CUs, and the cheap bricks come last,
    // where they fill the gaps.
    const int n_listed = table[0] + table[cap_ids + 1];
    const float tau = K.d_dt && !K.cell_scene ? (float)*K.d_dt : 0.0f;  // (the corrector's step)
    corrector_clock(K);
    // cell range (start, count) of staged cell t < S of brick b (count 0 for a
    // cell outside a non-periodic grid edge)
    auto ranges = [&](int b, int t, int &st, int &cnt) {
        const int cx0 = (b % G.nbx) * BX, cy0 = ((b / G.nbx) % G.nby) * BY, cz0 = (b / (G.nbx * G.nby)) * BZ;
        st = 0;
        cnt = 0;
        if (t < S) {
            int gx = cx0 - 1 + St::sx_of(t), gy = cy0 - 1 + St::sy_of(t), gz = cz0 - 1 + St::sz_of(t);
            const bool ok = wrap_axis(gx, G.nx, G.periodic & 1u) && wrap_axis(gy, G.ny, (G.periodic >> 1) & 1u) &&
                            wrap_axis(gz, G.nz, (G.periodic >> 2) & 1u);
            if (ok) {
                const int lin = gx + G.nx * (gy + G.ny * gz);
                st = cell_start[lin];
                cnt = cell_end[lin] - st;
            }
        }
    };
    // inner cell u of brick b holds centrals (inner cells past the grid edge
    // hold none: on a periodic axis the staged copy would be the wrapped cell,
    // owned by another brick)
    auto inner_in_grid = [&](int b, int u) {
        const int cx0 = (b % G.nbx) * BX, cy0 = ((b / G.nbx) % G.nby) * BY, cz0 = (b / (G.nbx * G.nby)) * BZ;
        return cx0 + St::ix_of(u) < G.nx && cy0 + St::iy_of(u) < G.ny && cz0 + St::iz_of(u) < G.nz;
    };
    // Scan ahead, by one wave: claim the next brick and write its cell scans
    // (the same values as the workgroup's block scans below) into buffer buf,
    // with wave operations only, while the other waves finish the current
    // brick's pairs.
    auto scan_ahead = [&](int lane, int buf) {
        int kb2 = 0;
        if (lane == 0) kb2 = atomicAdd(next, 1);
        kb2 = __shfl(kb2, 0);
        int total2 = 0, nc2 = 0;
        if (kb2 < n_listed) {
            const int b2 = brick_at(table, cap_ids, kb2);
            constexpr int NCH = (S + kWave - 1) / kWave;
            int st[NCH], ct[NCH], ex[NCH];
#pragma unroll
            for (int c = 0; c < NCH; ++c) ranges(b2, c * kWave + lane, st[c], ct[c]);
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                int inc = ct[c];
#pragma unroll
                for (int o = 1; o < kWave; o <<= 1) {
                    const int v = __shfl_up(inc, o);
                    if (lane >= o) inc += v;
                }
                ex[c] = total2 + inc - ct[c];
                const int t = c * kWave + lane;
                if (t < S) {
                    cBaseB[buf][t] = ex[c];
                    cDeltaB[buf][t] = ex[c] - st[c];
                }
                total2 += __shfl(inc, kWave - 1);
            }
            if (lane == 0) cBaseB[buf][S] = total2;
            // inner cell `lane`: the count and start of its staged cell, taken
            // from the lane that scanned it
            const int t = St::inner(min(lane, NI - 1));
            int vct = 0, vst = 0;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int a = __shfl(ct[c], t % kWave), s2 = __shfl(st[c], t % kWave);
                if (t / kWave == c) {
                    vct = a;
                    vst = s2;
                }
            }
            const int icnt = lane < NI && inner_in_grid(b2, lane) ? vct : 0;
            int inc = icnt;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const int v = __shfl_up(inc, o);
                if (lane >= o) inc += v;
            }
            nc2 = __shfl(inc, kWave - 1);
            if (lane < NI) {
                iBaseB[buf][lane] = inc - icnt;
                iStartB[buf][lane] = vst;
            }
            if (lane == 0) iBaseB[buf][NI] = nc2;
        }
        if (lane == 0) {
            sPre[1] = kb2;
            sPre[2] = total2;
            sPre[3] = nc2;
        }
    };
    int cur = 0;       // buffer of the current brick's scans
    bool pre = false;  // uniform: they were scanned ahead
    for (;;) {
        // the thread index is re-read per brick (an empty asm hides that it is
        // the same), so nothing derived from it is kept live across the pair loop
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        int kb, total, nc;
        if (pre) {
            kb = sPre[1];
            total = sPre[2];
            nc = sPre[3];
        } else {
            if (tid == 0) sNext = atomicAdd(next, 1);
            __syncthreads();
            kb = sNext;
        }
        if (kb >= n_listed) break;  // uniform
        const int b = brick_at(table, cap_ids, kb);
        const int cx0 = (b % G.nbx) * BX, cy0 = ((b / G.nbx) % G.nby) * BY, cz0 = (b / (G.nbx * G.nby)) * BZ;
        int *cBase = cBaseB[cur], *cDelta = cDeltaB[cur], *iBase = iBaseB[cur], *iStart = iStartB[cur];

        if (!pre) {
            // 1. ranges of the staged cells and their LDS bases (the staging
            //    order of the list build)
            int st, cnt;
            ranges(b, tid, st, cnt);
            const int ex = block_scan<NT>(cnt, total, wsum);
            if (tid < S) {
                cBase[tid] = ex;
                cDelta[tid] = ex - st;
            }
            if (tid == 0) cBase[S] = total;
            __syncthreads();
            // inner cells (x fastest: each inner row is one contiguous particle range)
            int icnt = 0, ist = 0;
            if (tid < NI && inner_in_grid(b, tid)) {
                const int t = St::inner(tid);
                icnt = cBase[t + 1] - cBase[t];
                ist = cBase[t] - cDelta[t];
            }
            const int iex = block_scan<NT>(icnt, nc, wsum);
            if (tid < NI) {
                iBase[tid] = iex;
                iStart[tid] = ist;
            }
            if (tid == 0) iBase[NI] = nc;
        }
        if (nc == 0) {  // uniform: no particle in the brick
            pre = false;
            __syncthreads();
            continue;
        }
        __syncthreads();
        const bool use_lds = total <= CAP;
        if (K.cell_scene && tid < NI) {
            // the step of each inner cell's scene, for the corrector of its
            // centrals (read after the staging barrier)
            int sc = -1;
            if (inner_in_grid(b, tid)) {
                const int lin = (cx0 + St::ix_of(tid)) +
                                G.nx * ((cy0 + St::iy_of(tid)) + G.ny * (cz0 + St::iz_of(tid)));
                sc = K.cell_scene[lin];
                if ((unsigned)sc >= (unsigned)K.n_scenes) sc = -1;
            }
            sSc[tid] = sc;
            sTau[tid] = sc >= 0 ? (float)K.d_dt[sc] : 0.0f;
        }
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
        // two lanes per central particle (lanes 2q', 2q' + 1): a brick holds
        // fewer centrals than the workgroup has lanes (about 840 at lattice
        // density), and half lists spread the work over all 16 waves
        const int h = tid & 1;
        if (tid == 0) sGroup = 0;  // read after the staging barrier
        // the list count of each wave's first group is requested before the staging loads
        // so the two latencies overlap (consecutive centrals stay on consecutive
        // lanes: their list groups are contiguous, one coalesced load per wave)
        int u0, i0;
        central(min(tid / 2, nc - 1), u0, i0);
        const uint32_t cnt0 = tid / 2 < nc ? count[i0] : 0u;
        if (use_lds) {
            // 2. stage the brick and its halo.  Wave w takes the staged rows w,
            //    w + NW, ... (a row is SX x-consecutive cells: one contiguous
            //    LDS range and, away from a periodic seam, one contiguous
            //    global range); the wave walks its rows as one range in chunks
            //    of 64 particles, the loads of SB chunks issued before their
            //    LDS stores so that their latencies overlap
            constexpr int NW = NT / kWave, NR = SY * SZ, RPW = (NR + NW - 1) / NW, SB = 4;
            const int wave = tid / kWave, lane = tid % kWave;
            int dlt[RPW], off[RPW + 1], e[RPW][SX - 1];
            off[0] = 0;
#pragma unroll
            for (int k = 0; k < RPW; ++k) {
                const int r = wave + k * NW, rr = min(r, NR - 1);
                const int b0 = cBase[rr * SX];
                dlt[k] = b0 - off[k];
                off[k + 1] = off[k] + (r < NR ? cBase[rr * SX + SX] - b0 : 0);
#pragma unroll
                for (int m = 0; m < SX - 1; ++m) e[k][m] = cBase[rr * SX + 1 + m];
            }
            const int L = off[RPW];
            for (int tb = 0; tb < L; tb += SB * kWave) {
                int slot[SB], cc[SB], rw[SB];
                float4 p[SB], v[SB];
                float ah[SB];  // alpha h of each loaded particle
                bool bnd[SB];
#pragma unroll
                for (int u = 0; u < SB; ++u) {
                    const int t = tb + u * kWave + lane;
                    int k = 0;
#pragma unroll
                    for (int m = 1; m < RPW; ++m) k += t >= off[m] ? 1 : 0;
                    int d = dlt[0], ee[SX - 1];
#pragma unroll
                    for (int m = 0; m < SX - 1; ++m) ee[m] = e[0][m];
#pragma unroll
                    for (int q = 1; q < RPW; ++q)
                        if (k == q) {
                            d = dlt[q];
#pragma unroll
                            for (int m = 0; m < SX - 1; ++m) ee[m] = e[q][m];
                        }
                    const int s2 = t + d;
                    int c = 0;
#pragma unroll
                    for (int m = 0; m < SX - 1; ++m) c += s2 >= ee[m] ? 1 : 0;
                    const int r = min(wave + k * NW, NR - 1);
                    slot[u] = t < L ? s2 : -1;
                    cc[u] = c;
                    rw[u] = r;
                    // past the wave's range a lane loads particle 0 (loads stay
                    // unconditional, so the chunk buffers stay in registers)
                    const int j = t < L ? s2 - cDelta[r * SX + c] : 0;
                    p[u] = pos[j];
                    v[u] = vel[j];
                    ah[u] = alpha_h_of(j, cell, C);
                    bnd[u] = (MODEL & kDiffusion) ? ptype(info[j]) == kBoundary : false;
                }
#pragma unroll
                for (int u = 0; u < SB; ++u) {
                    if (slot[u] >= 0) {
                        const float sx = (float)(cc[u] - 2), sy = (float)(rw[u] / SZ - 2),
                                    sz = (float)(rw[u] % SZ - 2);
                        // w = m x kernel coefficient, negated for boundary particles
                        // when the density diffusion needs the type
                        const float mf = p[u].w * C.fcoeff;
                        sP[slot[u]] = make_float4(fmaf(sx, C.csx, p[u].x), fmaf(sy, C.csy, p[u].y),
                                                  fmaf(sz, C.csz, p[u].z), bnd[u] ? -mf : mf);
                        sV[slot[u]] = v[u];
                        // equation-of-state terms from the staged density
                        sA[slot[u]] = eos_terms(v[u].w, ah[u], C);
                    }
                }
            }
        }
        __syncthreads();
        // (every thread read sPre at the top of this brick)
        if (tid == 0) sPre[0] = 0;

        // 3. two lanes per central particle of the brick, a wave taking
        //    kWave / 2 consecutive centrals at a time: wave w takes group w
        //    first (its counts were requested before the staging), then claims
        //    the next unclaimed group as it finishes one, so that waves that
        //    drew cheap groups (short lists) take more of the brick
        const int M = C.max_neibs;
        const uint32_t jmax = (uint32_t)(n - 1);
        constexpr int NW = NT / kWave, QG = kWave / 2;
        int g = tid / kWave;
        for (bool first = true; g * QG < nc; first = false) {  // wave-uniform
            const int q = g * QG + (tid % kWave) / 2;
            const bool act = q < nc;
            int u = u0, i = i0;
            uint32_t cntw = cnt0;
            if (!first) {
                central(act ? q : nc - 1, u, i);
                cntw = act ? count[i] : 0u;
            }
            const int nf = min((int)(cntw & 0xFFFFu), M);
            const int nt = min(nf + (int)(cntw >> 16), M);
            const int ntw = __builtin_amdgcn_readfirstlane(wave_max(nt));
            PairAcc A = {0.0f, 0.0f, 0.0f, 0.0f};
            float4 ustar;  // the central's own velocity (corrector stage)
            if (ntw > 0) {
                const size_t toff = (size_t)(i / kWave) * (kWave * M) + (i % kWave);
                if (use_lds) {
                    const int tc = St::inner(u);
                    const int si = i + cDelta[tc];
                    const uint4 *lg = (const uint4 *)(neibs_brick + brick_entry(i, 0, brick_groups(M)));
                    brick_pairs_lds<MODEL, NT>(A, lg, h, nt, ntw, total, sP, sV, sA, sP[si], sV[si], sA[si], C);
                    A.ax += __shfl_xor(A.ax, 1);
                    A.ay += __shfl_xor(A.ay, 1);
                    A.az += __shfl_xor(A.az, 1);
                    A.dr += __shfl_xor(A.dr, 1);
                    if (K.d_dt) ustar = sV[i + cDelta[St::inner(u)]];
                } else {
                    // the first lane of the pair walks the whole list (a shallow
                    // pipeline: this path shares the register budget of the LDS
                    // path and runs only where a halo overflows)
                    const bool central_fluid = (MODEL & kDiffusion) ? ptype(info[i]) != kBoundary : true;
                    const float4 vi = vel[i];
                    gather_pairs<MODEL, 2>(A, neibs + toff, nf, h == 0 ? nt : 0, ntw, M, jmax, pos, vel, nullptr, cell,
                                           pos[i], vi, eos_terms(vi.w, alpha_h_of(i, cell, C), C), central_fluid, C);
                    ustar = vi;
                }
            }
            // (particles with an empty list are written after the last brick)
            if (act && h == 0 && nt > 0) {
                const float4 f = make_float4(A.ax, A.ay, A.az, A.dr);
                if (out) out[i] = f;
                // (a central lies in one of the brick's cells: inner cell u)
                if (K.d_dt) {
                    if (!K.cell_scene)
                        corrector_apply(i, f, ustar, tau, K);
                    else if (sSc[u] >= 0)
                        corrector_apply(i, f, ustar, sTau[u], K);
                }
            }
            int gn = 0;
            if (tid % kWave == 0) gn = atomicAdd(&sGroup, 1) + NW;
            g = __builtin_amdgcn_readfirstlane(__shfl(gn, 0));
        }
        // the first wave left without a group scans the next brick ahead
        int won = 0;
        if (tid % kWave == 0) won = atomicCAS(&sPre[0], 0, 1) == 0;
        if (__builtin_amdgcn_readfirstlane(__shfl(won, 0))) scan_ahead(tid % kWave, cur ^ 1);
        __syncthreads();  // the next brick reuses the LDS
        pre = sPre[0] != 0;
        if (pre) cur ^= 1;
    }
    // Particles with an empty list (none of their bricks' pairs; also those
    // the build dropped) get zero derivatives, by all workgroups as they run
    // out of bricks: no other lane writes them.
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT)
        if (count[i] == 0u) {
            const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (out) out[i] = z;
            if (K.d_dt && K.cell[i] >= 0) corrector_at(i, z, vel[i], tau, K);
        }
}

// LDS capacity (staged particles, 40 bytes each) per brick shape: the halo
// of a brick at the h = 1.3 dp, r_s = 2.86 dp lattice density holds up to
// about 27 particles per staged cell (3 x 4 x 3: 150 cells, 3825 at most in
// the 1.62M dam break; 3 x 3 x 3: 125 cells, 3375; 3 x 2 x 3: 100 cells).
// Measured on the 1.62M dam break (one workgroup per CU in every case):
// 3 x 4 x 3 277 us, 3 x 3 x 3 357 us, 4 x 3 x 3 425 us (1% of its bricks
// overflow the LDS there).
constexpr int brick_cap(int BX, int BY, int BZ) { return BX * BY * BZ >= 36 ? 4000 : (BX * BY * BZ >= 27 ? 3400 : 2750); }

template <int MODEL>
void launch_brick(const ForceArgs &a, const ForceConst &C, hipStream_t s)
{
    with_shape(a.shape, [&]<int BX, int BY, int BZ>() {
        const BrickGrid G = brick_grid<BX, BY, BZ>(a.grid->ncell, a.grid->periodic);
        const unsigned blocks = (unsigned)G.nbx * G.nby * G.nbz;
        constexpr int NT = brick_threads(BX * BY * BZ);
        // (the brick counter was zeroed before the launch; the table of
        // bricks with a pair is the build's)
        const unsigned wgs = blocks < (unsigned)sph_device_cus() ? blocks : (unsigned)sph_device_cus();
        k_forces_brick<MODEL, BX, BY, BZ, NT, brick_cap(BX, BY, BZ)><<<wgs, NT, 0, s>>>(
            a.n, a.pos, a.vel, a.cell, a.neibs, a.neibs_brick, a.count, a.cell_start, a.cell_end, a.table,
            a.cap_ids, a.next, a.info, a.out, C, G, a.K);
    });
}

}  // namespace

#define SPH_PAIRS_FN_(k) forces_pairs_kernel##k
#define SPH_PAIRS_FN(k) SPH_PAIRS_FN_(k)

bool sph::SPH_PAIRS_FN(SPH_KERNEL_KIND)(int model, const ForceArgs &a, const ForceConst &C, hipStream_t s)
{
    if (model < 0 || model_kernel(model) != SPH_KERNEL_KIND) return false;
    return with_model<SPH_KERNEL_KIND>(model & kModelLowBits, [&]<int M>() {
        if (a.bricks) {
            // cell ranges and brick-local lists of the last build: LDS cell-brick
            // kernel (it writes the derivatives of every particle, those with an
            // empty list and those dropped by the build after its last brick)
            launch_brick<M>(a, C, s);
        } else {
            k_forces<M><<<sph_blocks(a.n, kThreads), kThreads, 0, s>>>(a.n, a.pos, a.vel, a.aux, a.neibs, a.count,
                                                                       a.info, a.out, C, a.K);
        }
    });
}
