// Time derivatives of the WCSPH step ("forces"): continuity, Cole equation
// of state, golden-rule pressure gradient with Monaghan artificial or Morris
// laminar viscosity, Wendland C2 kernel (arXiv:2207.11328, eq. mass-cont-sph1,
// eq. ns-sph1, section "Minimizing complexity", listing l:ktemplate).
//
// One lane per central particle gathers over its split neighbour list.  The
// list is neighbour-major, so slot k of 64 consecutive centres is one
// coalesced 256-byte load; the neighbours' pos/vel gathers hit L2 because
// particles are sorted by cell.  Fluid and boundary segments are walked in a
// single loop (slot k < nf from the front, the rest from the back) so lanes
// with different fluid/boundary splits stay converged.
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
    int cap;
};

// Cole EOS for gamma = 7 in the expanded form P = B d (7 + 21d + 35d^2 +
// 35d^3 + 21d^4 + 7d^5 + d^6), d = (rho - rho0)/rho0, which keeps full
// relative accuracy near rho0; returns P/rho^2 and c = c0 (1 + d)^3.
__device__ __forceinline__ void eos(float rho, const ForceConst &C, float &p_over_rho2, float &c)
{
    const float d = (rho - C.rho0) * C.inv_rho0;
    float poly = 7.0f + d;
    poly = fmaf(poly, d, 21.0f);
    poly = fmaf(poly, d, 35.0f);
    poly = fmaf(poly, d, 35.0f);
    poly = fmaf(poly, d, 21.0f);
    poly = fmaf(poly, d, 7.0f);
    const float P = C.B * d * poly;
    const float inv_rho = __builtin_amdgcn_rcpf(rho);
    p_over_rho2 = P * inv_rho * inv_rho;
    const float a = 1.0f + d;
    c = C.c0 * a * a * a;
}

__device__ __forceinline__ float unpack_shift(uint32_t e, int axis, float cs)
{
    const float b = (float)((e >> (26 + 2 * axis)) & 3u);
    return fmaf(b, cs, -cs);  // (b - 1) * cs, exact
}

template <int VISC>
__global__ __launch_bounds__(kThreads) void k_forces(int n, const float4 *__restrict__ pos,
                                                     const float4 *__restrict__ vel,
                                                     const uint32_t *__restrict__ neibs,
                                                     const uint32_t *__restrict__ count,
                                                     float4 *__restrict__ out, ForceConst C)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t cnt = count[i];
    // counts and indices are clamped so that a stale or foreign list can give
    // wrong numbers but never an out-of-bounds access
    const int nf = min((int)(cnt & 0xFFFFu), C.max_neibs);
    const int nt = min(nf + (int)(cnt >> 16), C.max_neibs);
    const uint32_t jmax = (uint32_t)(n - 1);
    const float4 pi = pos[i];
    const float4 vi = vel[i];
    const float rhoi = vi.w;
    float pri, ci;
    eos(rhoi, C, pri, ci);
    float ax = 0.0f, ay = 0.0f, az = 0.0f, dr = 0.0f;
    const uint32_t *col = neibs + i;
    for (int k = 0; k < nt; ++k) {
        const int slot = k < nf ? k : C.max_neibs - 1 + nf - k;
        const uint32_t e = col[(size_t)slot * C.cap];
        const uint32_t j = min(e & kIndexMask, jmax);
        const float tx = unpack_shift(e, 0, C.csx);
        const float ty = unpack_shift(e, 1, C.csy);
        const float tz = unpack_shift(e, 2, C.csz);
        const float4 pj = pos[j];
        const float4 vj = vel[j];
        const float r2 = predicate_r2(pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, tx, ty, tz);
        if (r2 < C.lim2) {
            const float xx = tx + (pi.x - pj.x);
            const float xy = ty + (pi.y - pj.y);
            const float xz = tz + (pi.z - pj.z);
            const float r = __builtin_amdgcn_sqrtf(r2);
            const float qm2 = fmaf(r, C.inv_h, -2.0f);
            const float F = C.fcoeff * qm2 * qm2 * qm2;
            const float ux = vi.x - vj.x;
            const float uy = vi.y - vj.y;
            const float uz = vi.z - vj.z;
            const float udx = fmaf(ux, xx, fmaf(uy, xy, uz * xz));
            const float mF = pj.w * F;
            dr = fmaf(mF, udx, dr);
            const float rhoj = vj.w;
            float prj, cj;
            eos(rhoj, C, prj, cj);
            float visc = 0.0f;
            if (udx < 0.0f) {
                // -alpha h cbar udx / (rhobar (r2 + eps h^2)) with the two
                // halves of the averages cancelling
                const float den = (rhoi + rhoj) * (r2 + C.eps_h2);
                visc = -C.alpha_h * (ci + cj) * udx * __builtin_amdgcn_rcpf(den);
            }
            const float coef = -mF * (pri + prj + visc);
            ax = fmaf(coef, xx, ax);
            ay = fmaf(coef, xy, ay);
            az = fmaf(coef, xz, az);
            if (VISC == 1) {
                const float lam = C.four_nu * mF * __builtin_amdgcn_rcpf(rhoi + rhoj);
                ax = fmaf(lam, ux, ax);
                ay = fmaf(lam, uy, ay);
                az = fmaf(lam, uz, az);
            }
        }
    }
    out[i] = make_float4(ax, ay, az, dr);
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
        const uint32_t cnt = count[i];
        const int nf = min((int)(cnt & 0xFFFFu), C.max_neibs);
        const int nt = min(nf + (int)(cnt >> 16), C.max_neibs);
        const uint32_t jmax = (uint32_t)(n - 1);
        const float4 pi = pos[i];
        for (int k = 0; k < nt; ++k) {
            const int slot = k < nf ? k : C.max_neibs - 1 + nf - k;
            const uint32_t e = neibs[(size_t)slot * C.cap + i];
            const float4 pj = pos[min(e & kIndexMask, jmax)];
            const float r2 = predicate_r2(pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, unpack_shift(e, 0, C.csx),
                                          unpack_shift(e, 1, C.csy), unpack_shift(e, 2, C.csz));
            c += r2 < C.lim2 ? 1ull : 0ull;
        }
    }
    c = wave_sum(c);
    if ((threadIdx.x % kWave) == 0 && c) atomicAdd(total, c);
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

bool make_const(const sph_grid *g, const sph_params *p, const sph_particles *parts, int max_neibs,
                ForceConst &C)
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
    C.cap = parts->capacity;
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

}  // namespace

extern "C" sph_status sph_forces(const sph_grid *grid, const sph_params *params, const sph_particles *parts,
                                 const uint32_t *neibs, const uint32_t *neib_count, int32_t max_neibs,
                                 float *forces, void *stream)
{
    if (!common_args(grid, params, parts, neibs, neib_count, max_neibs)) return SPH_ERR_ARG;
    if (parts->n > 0 && !forces) return SPH_ERR_ARG;
    ForceConst C;
    if (!make_const(grid, params, parts, max_neibs, C)) return SPH_ERR_ARG;
    const int n = parts->n;
    if (n == 0) return SPH_OK;
    hipStream_t s = (hipStream_t)stream;
    const float4 *pos = (const float4 *)parts->pos;
    const float4 *vel = (const float4 *)parts->vel;
    float4 *out = (float4 *)forces;
    if (params->visc_model == 0)
        k_forces<0><<<sph_blocks(n, kThreads), kThreads, 0, s>>>(n, pos, vel, neibs, neib_count, out, C);
    else
        k_forces<1><<<sph_blocks(n, kThreads), kThreads, 0, s>>>(n, pos, vel, neibs, neib_count, out, C);
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
    if (!make_const(grid, params, parts, max_neibs, C)) return SPH_ERR_ARG;
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
