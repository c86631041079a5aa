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
    int landrini;     // the equation-of-state prologue stores P instead of P/rho^2
};

struct ForceArgs {
    const sph_grid *grid;
    int shape;  // brick shape index
    int n;
    const float4 *pos, *vel;
    const float2 *aux;  // (P/rho^2 or P, alpha h c / 2) per particle
    const uint32_t *neibs, *count, *info;
    const uint16_t *neibs_brick;
    const int32_t *cell_start, *cell_end;
    int32_t *active;  // bricks holding particles: count, then ids
    int32_t *next;    // brick counter of the persistent workgroups
    int32_t *light;   // count of the light bricks, listed from the back of active
    uint8_t *cell_flags;  // cells holding a particle with a non-empty list (set by the prologue)
    float4 *out;
    bool bricks;
};

// Launch the pair kernel of `model` (sph_model.h bits) on stream s; false if
// the model's kernel is not the one of the translation unit.
bool forces_pairs_kernel0(int model, const ForceArgs &a, const ForceConst &C, hipStream_t s);
bool forces_pairs_kernel1(int model, const ForceArgs &a, const ForceConst &C, hipStream_t s);
bool forces_pairs_kernel2(int model, const ForceArgs &a, const ForceConst &C, hipStream_t s);
bool forces_pairs_kernel3(int model, const ForceArgs &a, const ForceConst &C, hipStream_t s);

}  // namespace sph
