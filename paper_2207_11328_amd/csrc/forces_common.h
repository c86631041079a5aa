// Constants and launch arguments of the derivative kernels, shared by the
// entry points (forces.hip) and the per-kernel pair translation units
// (forces_pairs.hip, one object per smoothing kernel).
#pragma once

#include "sph_model.h"

namespace sph {

struct ForceConst {
    float csx, csy, csz;
    float rho0, inv_rho0, B, c0;
    float lim2;       // fl32(2h)^2: interaction iff r2 < lim2
    float inv_h, inv_h2;
    float fcoeff;     // kernel coefficient c of F = c f(q)
    float alpha_h;    // alpha * h
    float eps_h2;     // eps * h^2
    float four_nu;    // 4 nu (Morris)
    float k_four_nu;  // 4 K nu (Monaghan K form)
    float diff;       // 2 delta h c0 (density diffusion)
    int max_neibs;
    int landrini;     // the equation-of-state terms hold P instead of P/rho^2
    float h;          // smoothing length (per-cell alpha times h)
    const float *cell_alpha;  // per-cell artificial-viscosity coefficient, or null
    int cell_base;
};

// Cole equation of state for gamma = 7 in the expanded form P = B d (7 + 21d
// + 35d^2 + 35d^3 + 21d^4 + 7d^5 + d^6), d = (rho - rho0)/rho0 (exact
// expansion of (1 + d)^7 - 1, full relative accuracy near rho0), as the pair
// terms use it: (P/rho^2, or P for the Landrini-Morris formulation, and
// alpha h c / 2 with c = c0 (1 + d)^3).  One definition for every kernel that
// needs it, so both derivative forms see bit-identical values.
__device__ __forceinline__ float2 eos_terms(float rho, float alpha_h, const ForceConst &C)
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
    return make_float2(C.landrini ? P : P * inv_rho * inv_rho, 0.5f * alpha_h * (C.c0 * a * a * a));
}

// alpha h of particle j: the coefficient of its cell when a per-cell table is
// given, else the global one
__device__ __forceinline__ float alpha_h_of(int j, const int32_t *__restrict__ cell, const ForceConst &C)
{
    return C.cell_alpha ? C.cell_alpha[cell[j] - C.cell_base] * C.h : C.alpha_h;
}

// The corrector stage taken inside the derivative kernel
// (sph_forces_corrector, sph_forces_corrector_scenes): as the derivatives f
// of a particle of state * are finished, its state n is advanced in place by
// dt (midpoint_stage with the stage velocity u*).  d_dt == nullptr:
// derivatives only.  With cell_scene, d_dt and d_time hold one step and one
// clock per scene and a particle takes its cell's scene's step.
struct Corrector {
    const double *d_dt;
    float4 *pos, *vel;  // state n, overwritten by state n+1
    const int32_t *cell;
    const uint32_t *info;
    double *d_time;     // advanced by dt once per call (per scene), or null
    float gx, gy, gz;
    const int32_t *cell_scene;  // scene of each cell (index cell - cell_base), or null
    int cell_base, n_scenes;
};

// The update of particle i, which lies in a cell (a particle the build
// dropped, cell < 0, is never passed here: it stays as it is); tau = (float)
// dt, read once per kernel for one scene; with scenes the step of the
// particle's scene (a cell of no scene: the particle stays as it is).  Its
// loads do not wait on one another except for the scene's step.
__device__ __forceinline__ void corrector_apply(int i, const float4 &f, const float4 &ustar, float tau,
                                                const Corrector &K)
{
    float4 p = K.pos[i], v = K.vel[i];
    midpoint_stage(p, v, ustar, f, ptype(K.info[i]) == kBoundary, tau, K.gx, K.gy, K.gz);
    K.pos[i] = p;
    K.vel[i] = v;
}

__device__ __forceinline__ void corrector_at(int i, const float4 &f, const float4 &ustar, float tau,
                                             const Corrector &K)
{
    if (K.cell_scene) {
        const int sc = K.cell_scene[K.cell[i] - K.cell_base];
        if ((unsigned)sc >= (unsigned)K.n_scenes) return;
        tau = (float)K.d_dt[sc];
    }
    corrector_apply(i, f, ustar, tau, K);
}

// The clocks the corrector advances: by block 0 at the start of the kernel.
__device__ __forceinline__ void corrector_clock(const Corrector &K)
{
    if (!K.d_dt || !K.d_time || blockIdx.x != 0) return;
    if (K.cell_scene) {
        for (int k = threadIdx.x; k < K.n_scenes; k += blockDim.x) K.d_time[k] += K.d_dt[k];
    } else if (threadIdx.x == 0) {
        *K.d_time += *K.d_dt;
    }
}

struct ForceArgs {
    const sph_grid *grid;
    int shape;  // brick shape index
    int n;
    const float4 *pos, *vel;
    const float2 *aux;  // (P/rho^2 or P, alpha h c / 2) per particle (gather form)
    const int32_t *cell;
    const uint32_t *neibs, *count, *info;
    const uint16_t *neibs_brick;
    const int32_t *cell_start, *cell_end;
    const int32_t *table;  // bricks with a pair (brick_table layout), from the build
    int cap_ids;           // ids of the table
    int32_t *next;         // brick counter of the persistent workgroups (zeroed before the launch)
    float4 *out;  // may be null when K.d_dt is set
    bool bricks;
    Corrector K;
};

// Launch the pair kernel of `model` (sph_model.h bits) on stream s; false if
// the model's kernel is not the one of the translation unit.
bool forces_pairs_kernel0(int model, const ForceArgs &a, const ForceConst &C, hipStream_t s);
bool forces_pairs_kernel1(int model, const ForceArgs &a, const ForceConst &C, hipStream_t s);
bool forces_pairs_kernel2(int model, const ForceArgs &a, const ForceConst &C, hipStream_t s);
bool forces_pairs_kernel3(int model, const ForceArgs &a, const ForceConst &C, hipStream_t s);

}  // namespace sph
