// Adjoint of the derivative sums (sph_forces) with the neighbour lists held
// fixed: the pair loops, for the smoothing kernel SPH_KERNEL_KIND (compiled
// once per kernel, every formulation / laminar term / diffusion instance of
// that kernel in both kernel forms).
//
// Forward pair term of central c and neighbour n (r < 2h), x = x_c - x_n,
// u = u_c - u_n, w = u.x:
//   a_c    += -m_n (S_p + Pi) F x  [+ Lm u]  [+ Lk x]
//   Drho_c += W_c m_n F w           [+ density diffusion]
//   S_p = p_c + p_n (p = P/rho^2), W_c = 1 (golden rule, eq. mass-cont-sph1,
//         eq. ns-sph1) or S_p = (P_c + P_n)/(rho_c rho_n), W_c = rho_c/rho_n
//         (Landrini-Morris, eq. mass-cont-sph2, eq. ns-sph2)
//   Pi = K min(w, 0) / (r^2 + eps h^2),  K = -alpha h (c_c + c_n)/(rho_c + rho_n)
//   Lm = 4 nu m_n F/(rho_c + rho_n)  (Morris),
//   Lk = 4 K' nu m_n F w/((rho_c + rho_n)(r^2 + eps h^2))  (Monaghan's K form)
// (with the readings of the design notes).
//
// Atomic-free gather: the list is symmetric (the float32 predicate gives
// x_ji = -x_ij bit for bit), so particle i visits each partner j once and
// collects both its role as central (upstream abar_i, dbar_i) and its role as
// neighbour of j (upstream abar_j, dbar_j).  With
//   da = m_j abar_i - m_i abar_j,  dA = da.x,  dU = da.u,
//   sD = m_j W_i dbar_i + m_i W_j dbar_j   (W_i = rho_i/rho_j, W_j = rho_j/rho_i, or 1)
// the two roles combine into
//   dL/do_i   += -S F da - dA (S F'/r x + F act K (u/d - 2 w x/d^2)) + sD (F u + w F'/r x)
//                [+ 4 nu F'/(rs r) dU x]  [+ Q da + dA kr ((F'/r w - 2 F w/d) x + F u)]
//   dL/du_i   += -F act K/d dA x + sD F x                       [+ 4 nu F/rs da]  [+ dA kr F x]
//   dL/drho_i += -F (dS_p/drho_i + dPi/drho_i) dA               [- 4 nu F/rs^2 dU]  [- Q dA/rs]
//                [+ w F (dbar_i m_j/rho_j - dbar_j m_i rho_j/rho_i^2)  (Landrini-Morris)]
// with S = S_p + Pi, d = r^2 + eps h^2, rs = rho_i + rho_j, act = (w < 0),
// kr = 4 K' nu/(rs d), Q = kr F w.
// Parameter derivatives are taken from the central role only:
//   dL/dalpha += abar_i.x (-m_j F) Pi/alpha,  dL/dc0 += abar_i.x (-m_j F)(2 S_p + Pi)/c0,
//   dL/dnu    += abar_i.u 4 m_j F/rs  or  abar_i.x 4 K' m_j F w/(rs d).
#include <hip/hip_runtime.h>
#include <math.h>

#include "backward_common.h"

#ifndef SPH_KERNEL_KIND
#error "compile with SPH_KERNEL_KIND set to one of the SPH_KERNEL_* values"
#endif

using namespace sph;

namespace {

constexpr int kThreads = 256;

struct BackAcc {
    float ox, oy, oz, ux, uy, uz, r;
    float galpha, gc0, gnu;
};

// aux: xi = (p or P, c, dp/drho or dP/drho, dc/drho) of the central; xj = (p
// or P, c) of the neighbour.  pair_fluid: both are fluid (density diffusion).
// MASKED: a pair outside the support or past the list has F and F'/r set to
// zero and is accumulated anyway (every term is a finite factor times one of
// them, so it adds +-0; the LDS loop only stages real particles, so every
// factor is finite); otherwise a branch skips it.  The LDS loop takes the
// masked form except with density diffusion, whose longer pair body spills
// when it runs for every slot.
template <int MODEL, bool MASKED>
__device__ __forceinline__ void pair_adjoint_core(BackAcc &G, float xx, float xy, float xz, float mi,
                                                  const float4 &vi, const float4 &xi, const float4 &gi, float mj,
                                                  const float4 &vj, const float2 &xj, const float4 &gj, bool valid,
                                                  bool pair_fluid, const BackConst &C)
{
    constexpr int KER = model_kernel(MODEL);
    float r2;
    {
#pragma clang fp contract(off)
        r2 = (xx * xx + xy * xy) + xz * xz;
    }
    bool inter = valid && (r2 < C.lim2);
    if constexpr (KER == SPH_KERNEL_QUADRATIC) inter = inter && r2 > 0.0f;  // its F is unbounded at r = 0
    // 1/r from one reciprocal square root, r = r^2/r
    const float inv_r = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * inv_r;
    float F, Fp_r;  // F and F'(r)/r
    kernel_F_dF<KER>(C.fcoeff, r, r2, inv_r, C.inv_h, C.inv_h2, F, Fp_r);
    if (MASKED) {
        F = inter ? F : 0.0f;
        Fp_r = inter ? Fp_r : 0.0f;
    }
    const float ux = vi.x - vj.x, uy = vi.y - vj.y, uz = vi.z - vj.z;
    const float w = fmaf(ux, xx, fmaf(uy, xy, uz * xz));
    const float rs = vi.w + vj.w;
    const float dd = r2 + C.eps_h2;
    // 1/rs and 1/d from one reciprocal (a quarter-rate operation) of their
    // product (rs d >= 2 rho eps h^2, far from the float range's ends)
    const float inv_rsd = __builtin_amdgcn_rcpf(rs * dd);
    const float inv_rs = dd * inv_rsd;
    const float inv_d = rs * inv_rsd;
    const float csum = xi.y + xj.y;
    // Pi = -alpha h min(w, 0)/d (c_i + c_j)/rs = A B with A = -alpha h min(w, 0)/d
    // (zero for w >= 0, and so are Pi and its rho_i derivative) and B = csum/rs
    const float mwd = fminf(w, 0.0f) * inv_d;
    const float B = csum * inv_rs;
    const float A = -C.alpha_h * mwd;
    const float Pi = A * B;
    const float actK = w < 0.0f ? -C.alpha_h * B : 0.0f;
    // dPi/drho_i = A (dc_i/drho_i - B)/rs
    const float dPi_dri = A * (xi.w - B) * inv_rs;
    // 1/(rho_i rho_j), 1/rho_i and 1/rho_j from one reciprocal (Landrini-Morris;
    // the density diffusion alone takes them in its branch)
    [[maybe_unused]] float inv_rr = 0.0f, iri = 0.0f, irj = 0.0f;
    if constexpr (MODEL & kLandrini) {
        inv_rr = __builtin_amdgcn_rcpf(vi.w * vj.w);
        iri = vj.w * inv_rr;
        irj = vi.w * inv_rr;
    }
    // pressure factor S_p and dS_p/drho_i
    float Sp, dSp;
    if constexpr (MODEL & kLandrini) {
        Sp = (xi.x + xj.x) * inv_rr;
        dSp = (xi.z - Sp * vj.w) * inv_rr;  // (c_i^2 - S_p rho_j)/(rho_i rho_j)
    } else {
        Sp = xi.x + xj.x;
        dSp = xi.z;
    }
    const float S = Sp + Pi;
    // combined upstream of the two roles
    const float dax = mj * gi.x - mi * gj.x;
    const float day = mj * gi.y - mi * gj.y;
    const float daz = mj * gi.z - mi * gj.z;
    const float dA = fmaf(dax, xx, fmaf(day, xy, daz * xz));
    float sD;
    [[maybe_unused]] float inv_ri = 0.0f, inv_rj = 0.0f, wj = 0.0f;
    if constexpr (MODEL & kLandrini) {
        inv_ri = iri;
        inv_rj = irj;
        wj = vj.w * inv_ri;
        sD = fmaf(mj * gi.w, vi.w * inv_rj, mi * gj.w * wj);
    } else {
        sD = fmaf(mj, gi.w, mi * gj.w);
    }
    // d/do_i = ka da + kx x + ku u, d/du_i = ku x (+ the laminar terms)
    const float t = w * inv_d;
    const float cu = F * actK * inv_d;
    const float cx = fmaf(-2.0f * t, cu, S * Fp_r);  // S F'/r - 2 F actK w/d^2
    float kx = fmaf(-dA, cx, sD * w * Fp_r);
    float ku = fmaf(-dA, cu, sD * F);
    float ka = -S * F;
    [[maybe_unused]] float kr = 0.0f, Q = 0.0f, duu = 0.0f;
    if constexpr (model_visc(MODEL) == kMonaghanK) {
        kr = C.k_four_nu * inv_rs * inv_d;
        Q = kr * F * w;
        ka += Q;
        kx = fmaf(dA * kr, fmaf(Fp_r, w, -2.0f * F * t), kx);
        ku = fmaf(dA * kr, F, ku);
    }
    if constexpr (model_visc(MODEL) == kMorris) {
        duu = fmaf(dax, ux, fmaf(day, uy, daz * uz));
        kx = fmaf(C.four_nu * Fp_r * inv_rs, duu, kx);
    }
    // d/drho_i
    float gr = F * (dSp + dPi_dri) * -dA;
    if constexpr (model_visc(MODEL) == kMorris) gr = fmaf(-C.four_nu * F * inv_rs * inv_rs, duu, gr);
    if constexpr (model_visc(MODEL) == kMonaghanK) gr = fmaf(-Q * inv_rs, dA, gr);
    if constexpr (MODEL & kLandrini) gr = fmaf(w * F, fmaf(gi.w * mj, inv_rj, -gj.w * mi * wj * inv_ri), gr);
    // parameters (central role)
    const float AmF = fmaf(gi.x, xx, fmaf(gi.y, xy, gi.z * xz)) * (-mj * F);
    float ga = AmF * (-C.h * mwd * B);
    float gc = AmF * fmaf(2.0f, Sp, Pi) * C.inv_c0;
    float gn = 0.0f;
    if constexpr (model_visc(MODEL) == kMorris) gn = fmaf(gi.x, ux, fmaf(gi.y, uy, gi.z * uz)) * 4.0f * mj * F * inv_rs;
    if constexpr (model_visc(MODEL) == kMonaghanK)
        gn = fmaf(gi.x, xx, fmaf(gi.y, xy, gi.z * xz)) * (4.0f * kMonaghanKFactor) * mj * F * w * inv_rs * inv_d;
    if constexpr (MODEL & kDiffusion) {
        // density diffusion, term_ij = c m_j (rho_i - rho_j)/rho_j Gd(r) with
        // Gd = F r^2/(r^2 + eps h^2), c = 2 delta h c0; both roles combined:
        //   do_i   += c Gd'/r (rho_i - rho_j)(dbar_i m_j/rho_j - dbar_j m_i/rho_i) x
        //   drho_i += c Gd (dbar_i m_j/rho_j - dbar_j m_i rho_j/rho_i^2)
        //   dc0    += dbar_i term_ij / c0   (central role)
        if (pair_fluid) {
            if constexpr (!(MODEL & kLandrini)) {
                inv_rr = __builtin_amdgcn_rcpf(vi.w * vj.w);
                iri = vj.w * inv_rr;
                irj = vi.w * inv_rr;
            }
            const float Gd = F * r2 * inv_d;
            const float Gd_r = Fp_r * r2 * inv_d + 2.0f * F * C.eps_h2 * inv_d * inv_d;
            const float w1 = gi.w * mj * irj, w2 = gj.w * mi * iri;
            const float dr = vi.w - vj.w;
            kx = fmaf(C.diff * Gd_r * dr, w1 - w2, kx);
            gr = fmaf(C.diff * Gd, w1 - w2 * vj.w * iri, gr);
            gc = fmaf(w1 * C.diff * dr * Gd, C.inv_c0, gc);
        }
    }
    if (MASKED || inter) {
        G.ox = fmaf(ka, dax, fmaf(kx, xx, fmaf(ku, ux, G.ox)));
        G.oy = fmaf(ka, day, fmaf(kx, xy, fmaf(ku, uy, G.oy)));
        G.oz = fmaf(ka, daz, fmaf(kx, xz, fmaf(ku, uz, G.oz)));
        G.ux = fmaf(ku, xx, G.ux);
        G.uy = fmaf(ku, xy, G.uy);
        G.uz = fmaf(ku, xz, G.uz);
        if constexpr (model_visc(MODEL) == kMorris) {
            const float la = C.four_nu * F * inv_rs;
            G.ux = fmaf(la, dax, G.ux);
            G.uy = fmaf(la, day, G.uy);
            G.uz = fmaf(la, daz, G.uz);
        }
        G.r += gr;
        G.galpha += ga;
        G.gc0 += gc;
        G.gnu += gn;
    }
}

template <int MODEL>
__device__ __forceinline__ void pair_adjoint(BackAcc &G, uint32_t e, const float4 &pi, const float4 &vi,
                                             const float4 &xi, const float4 &gi, const float4 &pj,
                                             const float4 &vj, const float4 &xj, const float4 &gj, bool valid,
                                             bool pair_fluid, const BackConst &C)
{
    const float xx = fmaf(entry_k(e, 0), C.csx, pi.x - pj.x);
    const float xy = fmaf(entry_k(e, 1), C.csy, pi.y - pj.y);
    const float xz = fmaf(entry_k(e, 2), C.csz, pi.z - pj.z);
    pair_adjoint_core<MODEL, false>(G, xx, xy, xz, pi.w, vi, xi, gi, pj.w, vj, make_float2(xj.x, xj.y), gj, valid,
                            pair_fluid, C);
}

template <int MODEL>
__global__ __launch_bounds__(kThreads) void k_forces_backward(
    int n, const float4 *__restrict__ pos, const float4 *__restrict__ vel, const float4 *__restrict__ aux,
    const float4 *__restrict__ gforce, const uint32_t *__restrict__ neibs, const uint32_t *__restrict__ count,
    const uint32_t *__restrict__ info, float4 *__restrict__ gpos, float4 *__restrict__ gvel,
    double *__restrict__ partial, int accumulate, BackConst C)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    const int lane = threadIdx.x % kWave;
    const int ii = min(i, n - 1);
    const int M = C.max_neibs;
    const uint32_t cnt = i < n ? count[i] : 0u;
    const int nf = min((int)(cnt & 0xFFFFu), M);
    const int nt = min(nf + (int)(cnt >> 16), M);
    const int last = max(nt - 1, 0);
    const int ntw = __builtin_amdgcn_readfirstlane(wave_max(nt));
    const uint32_t jmax = (uint32_t)(n - 1);
    BackAcc G = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (ntw > 0) {
        const int tile_id = __builtin_amdgcn_readfirstlane(i / kWave);
        const uint32_t *tile = neibs + (size_t)tile_id * (kWave * M);
        const float4 pi = pos[ii], vi = vel[ii], xi = aux[ii], gi = gforce[ii];
        const bool central_fluid = (MODEL & kDiffusion) ? ptype(info[ii]) != kBoundary : true;
        uint32_t eA = tile[list_slot(0, nf, last, M) * kWave + lane];
        uint32_t eNext = tile[list_slot(1, nf, last, M) * kWave + lane];
        uint32_t jA = min(eA & kIndexMask, jmax);
        float4 pA = pos[jA], vA = vel[jA], xA = aux[jA], gA = gforce[jA];
        for (int k = 0; k < ntw; k += 2) {
            const uint32_t eN2 = tile[list_slot(k + 2, nf, last, M) * kWave + lane];
            const uint32_t eB = eNext;
            const uint32_t jB = min(eB & kIndexMask, jmax);
            const float4 pB = pos[jB], vB = vel[jB], xB = aux[jB], gB = gforce[jB];
            pair_adjoint<MODEL>(G, eA, pi, vi, xi, gi, pA, vA, xA, gA, k < nt, central_fluid && k < nf, C);
            eNext = tile[list_slot(k + 3, nf, last, M) * kWave + lane];
            eA = eN2;
            jA = min(eA & kIndexMask, jmax);
            pA = pos[jA];
            vA = vel[jA];
            xA = aux[jA];
            gA = gforce[jA];
            pair_adjoint<MODEL>(G, eB, pi, vi, xi, gi, pB, vB, xB, gB, k + 1 < nt, central_fluid && k + 1 < nf,
                               C);
        }
    }
    if (i < n) {
        float4 po = make_float4(G.ox, G.oy, G.oz, 0.0f);
        float4 vo = make_float4(G.ux, G.uy, G.uz, G.r);
        if (nt == 0) po = vo = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (accumulate) {
            const float4 p0 = gpos[i], v0 = gvel[i];
            po = make_float4(p0.x + po.x, p0.y + po.y, p0.z + po.z, p0.w);
            vo = make_float4(v0.x + vo.x, v0.y + vo.y, v0.z + vo.z, v0.w + vo.w);
        } else {
            po.w = gpos[i].w;
        }
        gpos[i] = po;
        gvel[i] = vo;
    }
    // parameter derivatives: per-block partial sums in double, fixed order
    double a = nt > 0 ? (double)G.galpha : 0.0, c = nt > 0 ? (double)G.gc0 : 0.0,
           v = nt > 0 ? (double)G.gnu : 0.0;
    if (i >= n) a = c = v = 0.0;
    a = wave_sum(a);
    c = wave_sum(c);
    v = wave_sum(v);
    __shared__ double red[3][kThreads / kWave];
    const int w = threadIdx.x / kWave;
    if (lane == 0) {
        red[0][w] = a;
        red[1][w] = c;
        red[2][w] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int k = 0; k < kThreads / kWave; ++k) s += red[threadIdx.x][k];
        partial[3 * (size_t)blockIdx.x + threadIdx.x] = s;
    }
}

// Output of one particle's adjoint (overwrite or accumulate; grad_pos.w is
// left as it is).
__device__ __forceinline__ void store_adjoint(int i, int nt, const BackAcc &G, float4 *__restrict__ gpos,
                                              float4 *__restrict__ gvel, int accumulate)
{
    float4 po = make_float4(G.ox, G.oy, G.oz, 0.0f);
    float4 vo = make_float4(G.ux, G.uy, G.uz, G.r);
    if (nt == 0) po = vo = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const float4 p0 = gpos[i];
    if (accumulate) {
        const float4 v0 = gvel[i];
        po = make_float4(p0.x + po.x, p0.y + po.y, p0.z + po.z, p0.w);
        vo = make_float4(v0.x + vo.x, v0.y + vo.y, v0.z + vo.z, v0.w + vo.w);
    } else {
        po.w = p0.w;
    }
    gpos[i] = po;
    gvel[i] = vo;
}

// ---------------------------------------------------------------------------
// Cell-brick form of the adjoint (the cell perspective of section "Changing
// perspective: from the particle to the cell", as in sph_forces).  A brick of
// cells is processed in its lower and its upper half along y: the staging
// order puts y outermost, so the staged cells of a half (its inner rows and
// one halo row on each side) are one contiguous range of staging slots, and
// the brick-local list entries of its particles index into that range.  Per
// staged particle 56 bytes go to LDS (brick-relative position and mass,
// velocity and density, P/rho^2 and c, the upstream adjoint), which holds the
// halo of a half brick at the lattice density; a half that does not fit reads
// the global lists and arrays as k_forces_backward does.  The sums per pair
// are those of k_forces_backward; the separation is taken from brick-relative
// positions (rounding differs from the gather kernel at the ulp level).
#ifndef SPH_BACK_RING
#define SPH_BACK_RING 2
#endif
constexpr int kBackBrickThreads = 1024;
constexpr int kBackBrickCap = 2880;

// Pairs of one central's brick-local list, read from LDS, shared by two
// lanes: lane h of the pair takes the groups of 8 entries h, h + 2, h + 4, ...
// (list groups requested two iterations ahead, staged data R pairs ahead).
template <int MODEL>
__device__ __forceinline__ void brick_adjoint_lds(BackAcc &G, const uint4 *lg, int h, int nt, int ntw, int s_lo,
                                                  int span, const float4 *__restrict__ sP,
                                                  const float4 *__restrict__ sV, const float2 *__restrict__ sX,
                                                  const float4 *__restrict__ sG, const float4 &pi, const float4 &vi,
                                                  const float4 &xi, const float4 &gi, const BackConst &C)
{
    // pairs of staged data in flight; one for the longest pair bodies
    // (Landrini-Morris with density diffusion and a laminar term), which
    // would otherwise exceed the 128 registers of a 1024-lane workgroup
    constexpr bool kHeaviest = (MODEL & kLandrini) && (MODEL & kDiffusion) && model_visc(MODEL) != 0;
    constexpr int R = kHeaviest ? 1 : SPH_BACK_RING;
    const int lastg = max(nt - 1, 0) / kBrickGroup;
    const uint32_t smax = (uint32_t)(span - 1);
    float4 P[R], V[R], Gj[R];
    float2 X[R];
    auto fetch = [&](uint32_t slot, int r) {
        const uint32_t sl = min(slot - (uint32_t)s_lo, smax);  // stays inside the staged range
        P[r] = sP[sl];
        V[r] = sV[sl];
        X[r] = sX[sl];
        Gj[r] = sG[sl];
    };
    uint4 gc = lg[min(h, lastg) * kWave];
    uint4 gn = lg[min(h + 2, lastg) * kWave];
#pragma unroll
    for (int r = 0; r < R; ++r) fetch(group_entry(gc, r), r);
    for (int k = 0; k < ntw; k += 2 * kBrickGroup) {
        const int g0 = k / kBrickGroup + h;  // this lane's group
        const uint4 gnn = lg[min(g0 + 4, lastg) * kWave];
        const int rem = nt - g0 * kBrickGroup;  // entries of the list from this group on
#pragma unroll
        for (int s = 0; s < kBrickGroup; ++s) {
            const int r = s % R;
            // staged w = +-m_j, negative for boundary particles
            pair_adjoint_core<MODEL, !(MODEL & kDiffusion)>(G, pi.x - P[r].x, pi.y - P[r].y, pi.z - P[r].z, fabsf(pi.w), vi, xi, gi,
                                    fabsf(P[r].w), V[r], X[r], Gj[r], s < rem,
                                    pi.w > 0.0f && P[r].w > 0.0f, C);
            const int s2 = s + R;
            fetch(s2 < kBrickGroup ? group_entry(gc, s2) : group_entry(gn, s2 - kBrickGroup), r);
        }
        gc = gn;
        gn = gnn;
    }
}

__device__ __forceinline__ void add_partner(BackAcc &A)
{
    A.ox += __shfl_xor(A.ox, 1);
    A.oy += __shfl_xor(A.oy, 1);
    A.oz += __shfl_xor(A.oz, 1);
    A.ux += __shfl_xor(A.ux, 1);
    A.uy += __shfl_xor(A.uy, 1);
    A.uz += __shfl_xor(A.uz, 1);
    A.r += __shfl_xor(A.r, 1);
    A.galpha += __shfl_xor(A.galpha, 1);
    A.gc0 += __shfl_xor(A.gc0, 1);
    A.gnu += __shfl_xor(A.gnu, 1);
}

template <int MODEL, int BX, int BY, int BZ, int NT, int CAP>
__global__ __launch_bounds__(NT) void k_forces_backward_brick(
    int n, const float4 *__restrict__ pos, const float4 *__restrict__ vel,
    const float4 *__restrict__ gforce, const uint32_t *__restrict__ neibs, const uint16_t *__restrict__ neibs_brick,
    const uint32_t *__restrict__ count, const int32_t *__restrict__ cell_start, const int32_t *__restrict__ cell_end,
    const int32_t *__restrict__ table, int cap_ids, int32_t *__restrict__ next,
    const uint32_t *__restrict__ info,
    float4 *__restrict__ gpos, float4 *__restrict__ gvel, double *__restrict__ partial,
    double *__restrict__ grad_params, int accumulate, BackConst C, BrickGrid G)
{
    using St = Staging<BX, BY, BZ>;
    constexpr int SX = St::SX, SZ = St::SZ, S = St::S, NI = St::NI;
    constexpr int ROW = SX * SZ;       // staged cells per y row
    constexpr int IROW = BX * BZ;      // inner cells per y row
    constexpr int HALF = BY / 2;       // inner y rows of the lower half
    static_assert(S <= NT, "one thread per staged cell");
    __shared__ float4 sP[CAP];
    __shared__ float4 sV[CAP];
    __shared__ float2 sX[CAP];
    __shared__ float4 sG[CAP];
    __shared__ int cBase[S + 1];
    __shared__ int cDelta[S];
    __shared__ int iBase[NI + 1];
    __shared__ int iStart[NI];
    __shared__ int wsum[NT / kWave];
    __shared__ double red[3][NT / kWave];

    __shared__ int sNext;
    __shared__ int sLast;
    // One resident workgroup per CU takes the bricks with a pair one at a time
    // from the counter `next`, heavy ones first (brick_at order; no workgroup
    // for an empty brick; costs even out across CUs, cheap bricks come last).
    const int n_listed = table[0] + table[cap_ids + 1];
    for (;;) {
        // the thread index is re-read per brick (an empty asm hides that it is the
        // same), so nothing derived from it is kept live across the pair loop
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        if (tid == 0) sNext = atomicAdd(next, 1);
        __syncthreads();
        const int kb = sNext;
        if (kb >= n_listed) break;  // uniform
        const int b = brick_at(table, cap_ids, kb);
        const int cx0 = (b % G.nbx) * BX, cy0 = ((b / G.nbx) % G.nby) * BY, cz0 = (b / (G.nbx * G.nby)) * BZ;

        // 1. staged cell ranges and LDS bases, inner cells and their centrals
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
        int icnt = 0, ist = 0;
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
        __syncthreads();

        const int M = C.max_neibs;
        const int groups = brick_groups(M);
        const uint32_t jmax = (uint32_t)(n - 1);
        if (tid % kWave == 0) {  // this wave's parameter sums of the brick (only its lane 0 touches them)
            red[0][tid / kWave] = 0.0;
            red[1][tid / kWave] = 0.0;
            red[2][tid / kWave] = 0.0;
        }
        for (int half = 0; half < 2; ++half) {
            // inner rows [y0, y1), staged rows [y0, y1 + 2)
            const int y0 = half ? HALF : 0, y1 = half ? BY : HALF;
            const int s_lo = cBase[y0 * ROW];
            const int s_hi = cBase[(y1 + 2) * ROW];
            const int q_lo = iBase[y0 * IROW];
            const int q_hi = iBase[y1 * IROW];
            const int span = s_hi - s_lo;
            const bool use_lds = span <= CAP;
            if (use_lds && q_hi > q_lo) {
                // stage the half.  Wave w takes the staged rows R0 + w, R0 + w +
                // NW, ... (SX x-consecutive cells: contiguous in LDS) and walks
                // them as one range in chunks of 64 particles, the loads of SB
                // chunks issued before their LDS stores so that their
                // latencies overlap; lanes past the range load particle 0
                constexpr int NW = NT / kWave, RPW = ((BY - HALF + 2) * SZ + NW - 1) / NW, SB = 4;
                const int wave = tid / kWave, lane = tid % kWave;
                const int R0 = y0 * SZ, R1 = (y1 + 2) * SZ;
                int dlt[RPW], off[RPW + 1], e[RPW][SX - 1];
                off[0] = 0;
#pragma unroll
                for (int k = 0; k < RPW; ++k) {
                    const int r = R0 + wave + k * NW, rr = min(r, R1 - 1);
                    const int b0 = cBase[rr * SX];
                    dlt[k] = b0 - off[k];
                    off[k + 1] = off[k] + (r < R1 ? cBase[rr * SX + SX] - b0 : 0);
#pragma unroll
                    for (int m = 0; m < SX - 1; ++m) e[k][m] = cBase[rr * SX + 1 + m];
                }
                const int L = off[RPW];
                for (int tb = 0; tb < L; tb += SB * kWave) {
                    int slot[SB], cc[SB], rw[SB];
                    float4 p[SB], v[SB], g[SB];
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
                        const int r = min(R0 + wave + k * NW, R1 - 1);
                        slot[u] = t < L ? s2 : -1;
                        cc[u] = c;
                        rw[u] = r;
                        const int j = t < L ? s2 - cDelta[r * SX + c] : 0;
                        p[u] = pos[j];
                        v[u] = vel[j];
                        g[u] = gforce[j];
                        // mass negated for boundary particles when the diffusion needs the type
                        bnd[u] = (MODEL & kDiffusion) ? ptype(info[j]) == kBoundary : false;
                    }
#pragma unroll
                    for (int u = 0; u < SB; ++u) {
                        if (slot[u] >= 0) {
                            const float sx = (float)(cc[u] - 2), sy = (float)(rw[u] / SZ - 2),
                                        sz = (float)(rw[u] % SZ - 2);
                            const int l = slot[u] - s_lo;
                            sP[l] = make_float4(fmaf(sx, C.csx, p[u].x), fmaf(sy, C.csy, p[u].y),
                                                fmaf(sz, C.csz, p[u].z), bnd[u] ? -p[u].w : p[u].w);
                            sV[l] = v[u];
                            // equation-of-state terms (P/rho^2 or P, c) from the staged density
                            const float4 x = eos_grad_terms(v[u].w, C);
                            sX[l] = make_float2(x.x, x.y);
                            sG[l] = g[u];
                        }
                    }
                }
            }
            __syncthreads();
            // two lanes per central particle of the half (lane pairs 2q', 2q'+1)
            const int h = tid & 1;
            if (q_hi == q_lo) continue;  // uniform
            for (int q0 = q_lo; q0 < q_hi; q0 += NT / 2) {
                const int q = q0 + tid / 2;
                const bool act = q < q_hi;
                int u;
                {
                    int lo = 0, hi = NI - 1;
                    const int qq = act ? q : q_hi - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (iBase[mid] <= qq) lo = mid;
                        else hi = mid - 1;
                    }
                    u = lo;
                }
                const int i = iStart[u] + ((act ? q : q_hi - 1) - iBase[u]);
                const uint32_t cntw = act ? count[i] : 0u;
                const int nf = min((int)(cntw & 0xFFFFu), M);
                const int nt = min(nf + (int)(cntw >> 16), M);
                const int ntw = __builtin_amdgcn_readfirstlane(wave_max(nt));
                BackAcc A = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
                if (ntw > 0) {
                    if (use_lds) {
                        const int si = i + cDelta[St::inner(u)] - s_lo;
                        const uint4 *lg = (const uint4 *)(neibs_brick + brick_entry(i, 0, groups));
                        const float4 vi = sV[si];
                        brick_adjoint_lds<MODEL>(A, lg, h, nt, ntw, s_lo, span, sP, sV, sX, sG, sP[si], vi,
                                                eos_grad_terms(vi.w, C), sG[si], C);
                    } else {
                        // the lane pair splits the list by parity of the entry
                        const uint32_t *tile = neibs + (size_t)(i / kWave) * (kWave * M) + (i % kWave);
                        const float4 pi = pos[i], vi = vel[i], gi = gforce[i];
                        const float4 xi = eos_grad_terms(vi.w, C);
                        const bool central_fluid = (MODEL & kDiffusion) ? ptype(info[i]) != kBoundary : true;
                        const int last = max(nt - 1, 0);
                        for (int k = h; k < ntw; k += 2) {
                            const uint32_t e = tile[list_slot(k, nf, last, M) * kWave];
                            const uint32_t j = min(e & kIndexMask, jmax);
                            const float4 vj = vel[j];
                            pair_adjoint<MODEL>(A, e, pi, vi, xi, gi, pos[j], vj, eos_grad_terms(vj.w, C),
                                               gforce[j], k < nt, central_fluid && k < nf, C);
                        }
                    }
                }
                add_partner(A);
                const bool own = act && h == 0 && nt > 0;
                // (a particle with an empty list is written after the last brick)
                if (own) store_adjoint(i, nt, A, gpos, gvel, accumulate);
                // parameter sums: per wave and group of centrals, in double,
                // added to the wave's LDS slot in a fixed order (no per-lane
                // double kept across the loop: registers are the pair loop's)
                const double ga = wave_sum(own ? (double)A.galpha : 0.0);
                const double gc = wave_sum(own ? (double)A.gc0 : 0.0);
                const double gn = wave_sum(own ? (double)A.gnu : 0.0);
                if (tid % kWave == 0) {
                    red[0][tid / kWave] += ga;
                    red[1][tid / kWave] += gc;
                    red[2][tid / kWave] += gn;
                }
            }
            __syncthreads();  // the next half reuses LDS
        }
        // parameter partial sums of the brick, fixed order, stored by brick id
        if (tid < 3) {
            double sum = 0.0;
            for (int k = 0; k < NT / kWave; ++k) sum += red[tid][k];
            partial[3 * (size_t)b + tid] = sum;
        }
        __syncthreads();  // the next brick reuses the LDS
    }
    // Particles with an empty list (none of their bricks' pairs; also those
    // the build dropped) get a zero adjoint when the call overwrites
    // (grad_pos.w is kept), by all workgroups as they run out of bricks: no
    // other lane writes them.
    if (!accumulate)
        for (int k = blockIdx.x * NT + threadIdx.x; k < n; k += gridDim.x * NT)
            if (count[k] == 0u) {
                gpos[k] = make_float4(0.0f, 0.0f, 0.0f, gpos[k].w);
                gvel[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
    // The last workgroup to finish sums the partials of every brick of the
    // grid (bricks without a pair hold the zero written before the launch)
    // in a fixed order: each workgroup makes its partials visible device-wide
    // before it counts itself finished (next[1]), and the last one takes that
    // count's view of memory before it reads them.
    // (the thread index is hidden from the compiler here as in the loop, so
    // that nothing derived from it is computed before the loop and kept live)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    if (tid == 0) {
        __threadfence();
        sLast = atomicAdd(&next[1], 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (sLast) {  // uniform
        __threadfence();
        sum_partials<NT>(tid, G.nbx * G.nby * G.nbz, partial, grad_params, accumulate, red);
    }
}

template <int MODEL>
void launch_backward_brick(const BackArgs &a, const BackConst &C, hipStream_t s, int &n_bricks)
{
    with_shape(a.shape, [&]<int BX, int BY, int BZ>() {
        const BrickGrid G = brick_grid<BX, BY, BZ>(a.grid->ncell, a.grid->periodic);
        const unsigned blocks = (unsigned)G.nbx * G.nby * G.nbz;
        n_bricks = (int)blocks;
        // (the brick counters and the per-brick parameter partials were
        // cleared before the launch; the table of bricks with a pair is the
        // build's)
        const unsigned wgs = blocks < (unsigned)sph_device_cus() ? blocks : (unsigned)sph_device_cus();
        k_forces_backward_brick<MODEL, BX, BY, BZ, kBackBrickThreads, kBackBrickCap>
            <<<wgs, kBackBrickThreads, 0, s>>>(a.n, a.pos, a.vel, a.gforce, a.neibs, a.neibs_brick,
                                              a.count, a.cell_start, a.cell_end, a.table, a.cap_ids, a.next, a.info,
                                              a.gpos,
                                              a.gvel, a.partial, a.grad_params, a.accumulate, C, G);
    });
}

}  // namespace

#define SPH_BACK_FN_(k) backward_pairs_kernel##k
#define SPH_BACK_FN(k) SPH_BACK_FN_(k)

bool sph::SPH_BACK_FN(SPH_KERNEL_KIND)(int model, const BackArgs &a, const BackConst &C, hipStream_t s,
                                      int &n_partials)
{
    if (model < 0 || model_kernel(model) != SPH_KERNEL_KIND) return false;
    return with_model<SPH_KERNEL_KIND>(model & kModelLowBits, [&]<int M>() {
        if (a.bricks) {
            // cell ranges and brick-local lists of the last build: LDS bricks,
            // one partial per brick of the grid
            launch_backward_brick<M>(a, C, s, n_partials);
        } else {
            const unsigned blocks = sph_blocks(a.n, kThreads);
            n_partials = (int)blocks;
            k_forces_backward<M><<<blocks, kThreads, 0, s>>>(a.n, a.pos, a.vel, a.aux, a.gforce, a.neibs, a.count,
                                                            a.info, a.gpos, a.gvel, a.partial, a.accumulate, C);
        }
    });
}
