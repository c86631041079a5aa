// Constants and launch arguments of the adjoint kernels, shared by the entry
// points (forces_backward.hip) and the per-kernel pair translation units
// (forces_backward_pairs.hip, one object per smoothing kernel).
#pragma once

#include "sph_model.h"

namespace sph {

struct BackConst {
    float csx, csy, csz;
    float rho0, inv_rho0, B, c0;
    float lim2, inv_h, inv_h2, fcoeff;
    float alpha_h, h, eps_h2, four_nu, k_four_nu, inv_c0;
    float diff;  // 2 delta h c0 (density diffusion)
    int max_neibs;
    int landrini;  // aux holds (P, c, c^2, dc/drho) instead of (P/rho^2, c, d(P/rho^2)/drho, dc/drho)
};

// Equation-of-state terms of the adjoint for gamma = 7 in the expanded Cole
// form: (P/rho^2, c, d(P/rho^2)/drho, dc/drho), or (P, c, dP/drho = c^2,
// dc/drho) for the Landrini-Morris formulation.  One definition for the
// gather form's prologue and the brick form's staging.
__device__ __forceinline__ float4 eos_grad_terms(float rho, const BackConst &C)
{
    const float d = (rho - C.rho0) * C.inv_rho0;
    float poly = 7.0f + d;
    poly = fmaf(poly, d, 21.0f);
    poly = fmaf(poly, d, 35.0f);
    poly = fmaf(poly, d, 35.0f);
    poly = fmaf(poly, d, 21.0f);
    poly = fmaf(poly, d, 7.0f);
    const float P = C.B * d * poly;
    const float inv_rho = __builtin_amdgcn_rcpf(rho);  // (hardware reciprocal, 1 ulp; no division sequence)
    const float a = 1.0f + d;
    const float c = C.c0 * a * a * a;
    const float p = P * inv_rho * inv_rho;
    if (C.landrini) return make_float4(P, c, c * c, 3.0f * c * inv_rho);
    return make_float4(p, c, (c * c * inv_rho - 2.0f * P * inv_rho * inv_rho) * inv_rho, 3.0f * c * inv_rho);
}

struct BackArgs {
    const sph_grid *grid;
    int shape, n;
    const float4 *pos, *vel, *aux, *gforce;
    const uint32_t *neibs, *count, *info;
    const uint16_t *neibs_brick;
    const int32_t *cell_start, *cell_end;
    const int32_t *table;  // bricks with a pair (brick_table layout), from the build
    int cap_ids;           // ids of the table
    int32_t *next;         // brick counter and finished workgroups of the persistent workgroups (zeroed before)
    float4 *gpos, *gvel;
    double *partial;  // per-block (gather) or per-brick parameter partials
    double *grad_params;  // (brick form) the last workgroup to finish sums the partials into it
    int accumulate;
    bool bricks;
};

// Sum of nparts parameter partials (3 doubles each) by the NT threads of one
// workgroup (tid: the thread's index) in a fixed order: thread t adds
// partials t, t + NT, ... in four
// running sums combined in a fixed order, then the waves' sums in wave order
// (red: 3 x NT/kWave doubles of LDS).  out = sum, or out + sum to accumulate.
template <int NT>
__device__ __forceinline__ void sum_partials(int tid, int nparts, const double *__restrict__ partial,
                                             double *__restrict__ out, int accumulate, double (*red)[NT / kWave])
{
    double s[3][4] = {};
    int b = tid;
    for (; b + 3 * NT < nparts; b += 4 * NT)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < 3; ++k) s[k][u] += partial[3 * (size_t)(b + u * NT) + k];
    for (; b < nparts; b += NT)
        for (int k = 0; k < 3; ++k) s[k][0] += partial[3 * (size_t)b + k];
    const int lane = tid % kWave, w = tid / kWave;
    for (int k = 0; k < 3; ++k) {
        const double t = wave_sum((s[k][0] + s[k][1]) + (s[k][2] + s[k][3]));
        if (lane == 0) red[k][w] = t;
    }
    __syncthreads();
    if (tid < 3) {
        double t = 0.0;
        for (int k = 0; k < NT / kWave; ++k) t += red[tid][k];
        out[tid] = accumulate ? out[tid] + t : t;
    }
}

// Launch the adjoint pair kernel of `model` on stream s and return the number
// of parameter partials it writes in n_partials; false if the model's kernel
// is not the one of the translation unit.
bool backward_pairs_kernel0(int model, const BackArgs &a, const BackConst &C, hipStream_t s, int &n_partials);
bool backward_pairs_kernel1(int model, const BackArgs &a, const BackConst &C, hipStream_t s, int &n_partials);
bool backward_pairs_kernel2(int model, const BackArgs &a, const BackConst &C, hipStream_t s, int &n_partials);
bool backward_pairs_kernel3(int model, const BackArgs &a, const BackConst &C, hipStream_t s, int &n_partials);

}  // namespace sph
