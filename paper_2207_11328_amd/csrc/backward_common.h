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

struct BackArgs {
    const sph_grid *grid;
    int shape, n;
    const float4 *pos, *vel, *aux, *gforce;
    const uint32_t *neibs, *count, *info;
    const uint16_t *neibs_brick;
    const int32_t *cell_start, *cell_end;
    const int32_t *table;  // bricks with a pair (brick_table layout), from the build
    int cap_ids;           // ids of the table
    int32_t *next;         // brick counter of the persistent workgroups
    float4 *gpos, *gvel;
    double *partial;  // per-block (gather) or per-brick parameter partials
    int accumulate;
    bool bricks;
};

// Launch the adjoint pair kernel of `model` on stream s and return the number
// of parameter partials it writes in n_partials; false if the model's kernel
// is not the one of the translation unit.
bool backward_pairs_kernel0(int model, const BackArgs &a, const BackConst &C, hipStream_t s, int &n_partials);
bool backward_pairs_kernel1(int model, const BackArgs &a, const BackConst &C, hipStream_t s, int &n_partials);
bool backward_pairs_kernel2(int model, const BackArgs &a, const BackConst &C, hipStream_t s, int &n_partials);
bool backward_pairs_kernel3(int model, const BackArgs &a, const BackConst &C, hipStream_t s, int &n_partials);

}  // namespace sph
