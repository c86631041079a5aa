// Adjoint of the derivative sums (sph_forces) with the neighbour lists held
// fixed, entry points: argument checks, the equation-of-state prologue of the
// gather form (the brick form takes the terms at staging), the
// dispatch to the pair kernels of the model (forces_backward_pairs.hip, one
// object per smoothing kernel), the fixed-order reduction of the parameter
// derivatives, and the permutation helper used to carry adjoints across a
// rebuild.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "backward_common.h"

using namespace sph;

namespace {

constexpr int kThreads = 256;

// Gather form: the equation-of-state terms of every particle, aux =
// eos_grad_terms(rho).  (The brick form evaluates them as it stages
// particles.)
__global__ __launch_bounds__(kThreads) void k_eos_grad(int n, const float4 *__restrict__ vel,
                                                       float4 *__restrict__ aux, BackConst C)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) aux[i] = eos_grad_terms(vel[i].w, C);
}

// Brick form: clears what the brick kernel counts and sums into, its two
// counters (next) and the nbp per-brick parameter partials.
__global__ __launch_bounds__(kThreads) void k_back_clear(int32_t *__restrict__ next, double *__restrict__ bpartial,
                                                         int nbp)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    for (int k = i; k < nbp; k += gridDim.x * kThreads) bpartial[k] = 0.0;
    if (i < 2) next[i] = 0;
}

// Sum of the per-block (or per-brick) parameter partials in a fixed order:
// thread t adds partials t, t + 1024, ... (four running sums, combined in a
// fixed order), then a fixed tree over the threads.
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void k_param_reduce(int nblocks, const double *__restrict__ partial,
                                                                 double *__restrict__ out, int accumulate)
{
    __shared__ double red[3][kReduceThreads / kWave];
    sum_partials<kReduceThreads>(threadIdx.x, nblocks, partial, out, accumulate, red);
}

__global__ __launch_bounds__(kThreads) void k_unpermute(int n, const uint32_t *__restrict__ perm,
                                                        const float4 *__restrict__ src, float4 *__restrict__ dst)
{
    const int k = blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    const uint32_t d = perm[k];
    if (d < (uint32_t)n) dst[d] = src[k];
}

size_t aux_bytes(int64_t cap) { return (size_t)((16 * cap + 255) & ~(int64_t)255); }
size_t partial_bytes(int64_t cap) { return (size_t)(3 * 8 * ((cap + kThreads - 1) / kThreads) + 256); }
// per-brick parameter partials (at most one brick per cell) and the brick
// counter
size_t brick_bytes(int64_t n_cells) { return (size_t)(3 * 8 * (n_cells + 1) + 256); }

}  // namespace

extern "C" size_t sph_forces_backward_workspace_bytes(int32_t capacity, int32_t n_cells)
{
    if (capacity < 0 || n_cells < 0) return 0;
    const int64_t cap = capacity > 0 ? capacity : 1;
    return aux_bytes(cap) + partial_bytes(cap) + brick_bytes(n_cells);
}

extern "C" sph_status sph_forces_backward(const sph_grid *grid, const sph_params *p, const sph_particles *parts,
                                          const uint32_t *neibs, const uint32_t *neib_count, int32_t max_neibs,
                                          const int32_t *cell_start, const int32_t *cell_end,
                                          const uint16_t *neibs_brick, const float *grad_forces, float *grad_pos,
                                          float *grad_vel, double *grad_params, int32_t accumulate,
                                          void *workspace, size_t workspace_bytes, void *stream)
{
    if (!grid || !p || !parts || !grad_params || grid->cell_alpha) return SPH_ERR_ARG;
    if (parts->n < 0 || parts->capacity < parts->n || parts->capacity > SPH_MAX_CAPACITY) return SPH_ERR_ARG;
    if (max_neibs < 1 || max_neibs > 65535) return SPH_ERR_ARG;
    if (parts->n > 0 && (!parts->pos || !parts->vel || !neibs || !neib_count || !grad_forces || !grad_pos ||
                         !grad_vel))
        return SPH_ERR_ARG;
    if (!(p->h > 0.0f) || !(p->rho0 > 0.0f) || !(p->c0 > 0.0f) || p->gamma != 7.0f) return SPH_ERR_ARG;
    if (model_of(p) < 0) return SPH_ERR_ARG;
    if (!(p->delta >= 0.0f) || !(p->delta < 1e30f)) return SPH_ERR_ARG;
    if (p->delta != 0.0f && parts->n > 0 && !parts->info) return SPH_ERR_ARG;
    const int64_t n_cells = (int64_t)grid->ncell[0] * grid->ncell[1] * grid->ncell[2];
    if (n_cells <= 0 || n_cells > INT32_MAX - 2) return SPH_ERR_ARG;
    const bool bricks = cell_start && cell_end && neibs_brick;
    const int shape = brick_shape_index(grid->brick);
    if (shape < 0) return SPH_ERR_ARG;
    if (bricks && parts->n > 0 && !parts->cell) return SPH_ERR_ARG;
    if (bricks && ((uintptr_t)neibs_brick & 15u)) return SPH_ERR_ARG;  // read in 16-byte groups
    if (!workspace || workspace_bytes < sph_forces_backward_workspace_bytes(parts->capacity, (int32_t)n_cells))
        return SPH_ERR_WORKSPACE;
    BackConst C;
    C.csx = grid->cell_size[0];
    C.csy = grid->cell_size[1];
    C.csz = grid->cell_size[2];
    C.rho0 = p->rho0;
    C.inv_rho0 = (float)(1.0 / (double)p->rho0);
    C.B = (float)((double)p->rho0 * (double)p->c0 * (double)p->c0 / (double)p->gamma);
    C.c0 = p->c0;
    const float two_h = 2.0f * p->h;
    C.lim2 = two_h * two_h;
    const double h = p->h;
    C.inv_h = (float)(1.0 / h);
    C.inv_h2 = (float)(1.0 / (h * h));
    C.fcoeff = (float)kernel_coeff(p->kernel, h);
    C.alpha_h = (float)((double)p->alpha * h);
    C.h = p->h;
    C.eps_h2 = (float)((double)p->eps_visc * h * h);
    C.four_nu = (float)(4.0 * (double)p->nu);
    C.k_four_nu = (float)(4.0 * (double)kMonaghanKFactor * (double)p->nu);
    C.inv_c0 = (float)(1.0 / (double)p->c0);
    C.diff = (float)(2.0 * (double)p->delta * h * (double)p->c0);
    C.max_neibs = max_neibs;
    C.landrini = p->formulation == SPH_FORM_LANDRINI_MORRIS;
    const int n = parts->n;
    hipStream_t s = (hipStream_t)stream;
    const int64_t cap1 = parts->capacity > 0 ? parts->capacity : 1;
    float4 *aux = (float4 *)workspace;
    double *partial = (double *)((char *)workspace + aux_bytes(cap1));
    double *bpartial = (double *)((char *)workspace + aux_bytes(cap1) + partial_bytes(cap1));
    int32_t *next = (int32_t *)(bpartial + 3 * (n_cells + 1));
    const int nblocks = n > 0 ? (int)sph_blocks(n, kThreads) : 0;
    static bool (*const pairs[4])(int, const BackArgs &, const BackConst &, hipStream_t, int &) = {
        backward_pairs_kernel0, backward_pairs_kernel1, backward_pairs_kernel2, backward_pairs_kernel3};
    const int model = model_of(p);
    int n_partials = 0;
    if (n > 0) {
        // bricks of the grid (one parameter partial each)
        int n_bricks = 0;
        with_shape(shape, [&]<int BX, int BY, int BZ>() {
            const BrickGrid G = brick_grid<BX, BY, BZ>(grid->ncell, grid->periodic);
            n_bricks = G.nbx * G.nby * G.nbz;
        });
        if (bricks) {
            const int nbp = 3 * n_bricks;
            const unsigned cb = (unsigned)std::min(std::max((nbp + kThreads - 1) / kThreads, 1), 256);
            k_back_clear<<<cb, kThreads, 0, s>>>(next, bpartial, nbp);
        } else {
            k_eos_grad<<<nblocks, kThreads, 0, s>>>(n, (const float4 *)parts->vel, aux, C);
        }
        BackArgs a;
        a.grid = grid;
        a.shape = shape;
        a.n = n;
        a.pos = (const float4 *)parts->pos;
        a.vel = (const float4 *)parts->vel;
        a.aux = aux;
        a.gforce = (const float4 *)grad_forces;
        a.neibs = neibs;
        a.count = neib_count;
        a.info = parts->info;
        a.neibs_brick = neibs_brick;
        a.cell_start = cell_start;
        a.cell_end = cell_end;
        a.cap_ids = brick_table_cap(parts->capacity);
        a.table = bricks ? brick_table(reinterpret_cast<const int32_t *>(neibs_brick), parts->capacity, max_neibs)
                         : nullptr;
        a.next = next;
        a.gpos = (float4 *)grad_pos;
        a.gvel = (float4 *)grad_vel;
        a.partial = bricks ? bpartial : partial;
        a.grad_params = grad_params;
        a.accumulate = accumulate;
        a.bricks = bricks;
        if (!pairs[model_kernel(model)](model, a, C, s, n_partials)) return SPH_ERR_ARG;
    }
    // (the brick kernel's last workgroup has summed the partials itself)
    if (!(bricks && n > 0))
        k_param_reduce<<<1, kReduceThreads, 0, s>>>(n_partials, partial, grad_params, accumulate);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

extern "C" sph_status sph_unpermute(int32_t n, const uint32_t *perm, const float *src, float *dst, void *stream)
{
    if (n < 0 || (n > 0 && (!perm || !src || !dst || src == dst))) return SPH_ERR_ARG;
    if (n == 0) return SPH_OK;
    k_unpermute<<<sph_blocks(n, kThreads), kThreads, 0, (hipStream_t)stream>>>(n, perm, (const float4 *)src,
                                                                              (float4 *)dst);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}
