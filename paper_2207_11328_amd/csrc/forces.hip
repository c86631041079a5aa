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

struct ForceConst {
    float csx, csy, csz;
    float rho0, inv_rho0, B, c0;
    float lim2;      // fl32(2h)^2: interaction iff r2 < lim2
    float inv_h;
    float fcoeff;    // 105 / (128 pi h^5)
    float alpha_h;   // alpha * h
    float eps_h2;    // eps * h^2
    float four_nu;   // 4 nu
    int max_neibs;
};

// Cole EOS for gamma = 7 in the expanded form P = B d (7 + 21d + 35d^2 +
// 35d^3 + 21d^4 + 7d^5 + d^6), d = (rho - rho0)/rho0 (exact expansion of
// (1 + d)^7 - 1, full relative accuracy near rho0).  aux = (P/rho^2, alpha h c)
// with c = c0 (1 + d)^3.
__global__ __launch_bounds__(kThreads) void k_eos(int n, const float4 *__restrict__ vel, float2 *__restrict__ aux,
                                                  const int32_t *__restrict__ cell,
                                                  const float *__restrict__ cell_alpha, int cell_base, float h,
                                                  ForceConst C)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    float alpha_h = C.alpha_h;
    if (cell_alpha) {
        const int c = cell[i];
        if (c >= 0) alpha_h = cell_alpha[c - cell_base] * h;
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
    aux[i] = make_float2(P * inv_rho * inv_rho, alpha_h * (C.c0 * a * a * a));
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

// One pair (i, j) of the derivative sums, branch-free; contributes only when
// `valid` (slot inside i's list) and r < 2h.
template <int VISC>
__device__ __forceinline__ void pair_terms(PairAcc &A, uint32_t e, const float4 &pi, const float4 &vi,
                                           const float2 &ai, const float4 &pj, const float4 &vj, const float2 &aj,
                                           bool valid, const ForceConst &C)
{
    // separation, bit-identical to the list predicate: x = k cs + (o_i - o_j)
    const float xx = fmaf(entry_k(e, 0), C.csx, pi.x - pj.x);
    const float xy = fmaf(entry_k(e, 1), C.csy, pi.y - pj.y);
    const float xz = fmaf(entry_k(e, 2), C.csz, pi.z - pj.z);
    float r2;
    {
#pragma clang fp contract(off)
        r2 = (xx * xx + xy * xy) + xz * xz;
    }
    const bool inter = valid && (r2 < C.lim2);
    const float r = __builtin_amdgcn_sqrtf(r2);
    const float qm2 = fmaf(r, C.inv_h, -2.0f);
    const float mF = (qm2 * qm2) * (qm2 * C.fcoeff) * pj.w;  // m_j F_ij
    const float ux = vi.x - vj.x;
    const float uy = vi.y - vj.y;
    const float uz = vi.z - vj.z;
    const float udx = fmaf(ux, xx, fmaf(uy, xy, uz * xz));
    A.dr = inter ? fmaf(mF, udx, A.dr) : A.dr;
    // Monaghan: Pi = -alpha h (c_i + c_j)/2 min(u.x, 0) / ((rho_i + rho_j)/2 (r^2 + eps h^2))
    const float den = (vi.w + vj.w) * (r2 + C.eps_h2);
    const float visc = -(ai.y + aj.y) * fminf(udx, 0.0f) * __builtin_amdgcn_rcpf(den);
    const float coef = inter ? -mF * (ai.x + aj.x + visc) : 0.0f;
    A.ax = fmaf(coef, xx, A.ax);
    A.ay = fmaf(coef, xy, A.ay);
    A.az = fmaf(coef, xz, A.az);
    if (VISC == 1) {
        const float lam = inter ? C.four_nu * mF * __builtin_amdgcn_rcpf(vi.w + vj.w) : 0.0f;
        A.ax = fmaf(lam, ux, A.ax);
        A.ay = fmaf(lam, uy, A.ay);
        A.az = fmaf(lam, uz, A.az);
    }
}

template <int VISC>
__global__ __launch_bounds__(kThreads) void k_forces(int n, const float4 *__restrict__ pos,
                                                     const float4 *__restrict__ vel,
                                                     const float2 *__restrict__ aux,
                                                     const uint32_t *__restrict__ neibs,
                                                     const uint32_t *__restrict__ count,
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
    const int last = max(nt - 1, 0);
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

    // Software pipeline, unrolled by two.  Entry k+2 is requested before pair k
    // is evaluated and the neighbour data of pair k+1 while pair k is being
    // evaluated; the data registers of set A are only ever written by loads,
    // so the loop carries no copy of an in-flight value.
    uint32_t eA = tile[list_slot(0, nf, last, M) * kWave + lane];
    uint32_t eNext = tile[list_slot(1, nf, last, M) * kWave + lane];
    uint32_t jA = min(eA & kIndexMask, jmax);
    float4 pA = pos[jA], vA = vel[jA];
    float2 xA = aux[jA];
    for (int k = 0; k < ntw; k += 2) {
        const uint32_t eN2 = tile[list_slot(k + 2, nf, last, M) * kWave + lane];
        const uint32_t eB = eNext;
        const uint32_t jB = min(eB & kIndexMask, jmax);
        const float4 pB = pos[jB], vB = vel[jB];
        const float2 xB = aux[jB];
        pair_terms<VISC>(A, eA, pi, vi, ai, pA, vA, xA, k < nt, C);
        eNext = tile[list_slot(k + 3, nf, last, M) * kWave + lane];
        eA = eN2;
        jA = min(eA & kIndexMask, jmax);
        pA = pos[jA];
        vA = vel[jA];
        xA = aux[jA];
        pair_terms<VISC>(A, eB, pi, vi, ai, pB, vB, xB, k + 1 < nt, C);
    }
    if (i < n) out[i] = nt > 0 ? make_float4(A.ax, A.ay, A.az, A.dr) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
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

extern "C" size_t sph_forces_workspace_bytes(int32_t capacity)
{
    if (capacity < 0) return 0;
    return aux_bytes(capacity > 0 ? capacity : 1);
}

extern "C" sph_status sph_forces(const sph_grid *grid, const sph_params *params, const sph_particles *parts,
                                 const uint32_t *neibs, const uint32_t *neib_count, int32_t max_neibs,
                                 float *forces, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!common_args(grid, params, parts, neibs, neib_count, max_neibs)) return SPH_ERR_ARG;
    if (parts->n > 0 && !forces) return SPH_ERR_ARG;
    ForceConst C;
    if (!make_const(grid, params, max_neibs, C)) return SPH_ERR_ARG;
    if (!workspace || workspace_bytes < sph_forces_workspace_bytes(parts->capacity)) return SPH_ERR_WORKSPACE;
    const int n = parts->n;
    if (n == 0) return SPH_OK;
    hipStream_t s = (hipStream_t)stream;
    const float4 *pos = (const float4 *)parts->pos;
    const float4 *vel = (const float4 *)parts->vel;
    float2 *aux = (float2 *)workspace;
    float4 *out = (float4 *)forces;
    if (grid->cell_alpha && !parts->cell) return SPH_ERR_ARG;
    k_eos<<<sph_blocks(n, kThreads), kThreads, 0, s>>>(n, vel, aux, parts->cell, grid->cell_alpha, grid->cell_base,
                                                       params->h, C);
    if (params->visc_model == 0)
        k_forces<0><<<sph_blocks(n, kThreads), kThreads, 0, s>>>(n, pos, vel, aux, neibs, neib_count, out, C);
    else
        k_forces<1><<<sph_blocks(n, kThreads), kThreads, 0, s>>>(n, pos, vel, aux, neibs, neib_count, out, C);
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
