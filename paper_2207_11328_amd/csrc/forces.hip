// Time derivatives of the WCSPH step ("forces"), entry points: argument
// checks, the equation-of-state prologue of the gather form, and the
// dispatch to the pair kernels of the model (arXiv:2207.11328, eq. mass-cont-sph1, eq. ns-sph1,
// eq. mass-cont-sph2, eq. ns-sph2, section "Minimizing complexity", listing
// l:ktemplate).  The pair loops live in forces_pairs.hip, one object per
// smoothing kernel.
//
// The gather form's prologue evaluates the equation of state once per
// particle (P/rho^2, or P for the Landrini-Morris formulation, and alpha h
// c), so its pair loop gathers 8 bytes instead of recomputing a 6th-order
// polynomial and a reciprocal per pair; the brick form evaluates the same
// terms as it stages particles in LDS.
#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>

#include "forces_common.h"

using namespace sph;

// Device scratch of the allocation-free entry point sph_forces_noalloc: it
// holds the workspace of sph_forces (equation-of-state terms, brick list and
// counters, cell flags) for problems whose sph_forces_workspace_bytes is at
// most SPH_NOALLOC_SCRATCH_BYTES.  Each device the library runs on holds its
// own copy from module load to the end of the process.  Host code never uses
// this name as an address: the device address comes from
// hipGetSymbolAddress, once per device (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[SPH_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kThreads = 256;

// Equation-of-state terms of the gather form (eos_terms): aux = (P/rho^2
// or P, alpha h c / 2) per particle.  The brick form evaluates them while it
// stages particles in LDS and needs no such pass.
__global__ __launch_bounds__(kThreads) void k_eos(int n, const float4 *__restrict__ vel, float2 *__restrict__ aux,
                                                  const int32_t *__restrict__ cell, ForceConst C)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const float alpha_h = C.cell_alpha && cell[i] >= 0 ? alpha_h_of(i, cell, C) : C.alpha_h;
    aux[i] = eos_terms(vel[i].w, alpha_h, C);
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

// the clocks advance by their steps (one per scene)
__global__ void k_add_time(double *d_time, const double *d_dt, int n_clocks)
{
    for (int k = threadIdx.x; k < n_clocks; k += blockDim.x) d_time[k] += d_dt[k];
}

// missed pairs of a rebuild: the difference of the two counts, and its running total
__global__ void k_missed_finish(long long *m)
{
    m[2] = m[1] - m[0];
    m[3] += m[2];
}

bool make_const(const sph_grid *g, const sph_params *p, int max_neibs, ForceConst &C)
{
    if (!(p->h > 0.0f) || !(p->rho0 > 0.0f) || !(p->c0 > 0.0f) || p->gamma != 7.0f) return false;
    if (model_of(p) < 0) return false;
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
    const double h = p->h;
    C.inv_h = (float)(1.0 / h);
    C.inv_h2 = (float)(1.0 / (h * h));
    C.fcoeff = (float)kernel_coeff(p->kernel, h);
    C.alpha_h = (float)((double)p->alpha * h);
    C.eps_h2 = (float)((double)p->eps_visc * h * h);
    C.four_nu = (float)(4.0 * (double)p->nu);
    C.k_four_nu = (float)(4.0 * (double)kMonaghanKFactor * (double)p->nu);
    C.diff = (float)(2.0 * (double)p->delta * h * (double)p->c0);
    C.max_neibs = max_neibs;
    C.landrini = p->formulation == SPH_FORM_LANDRINI_MORRIS;
    C.h = p->h;
    C.cell_alpha = g->cell_alpha;
    C.cell_base = g->cell_base;
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

// Device address of `scratch` on the current device, looked up on the first
// call on that device (with it current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

sph_status noalloc_scratch(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SPH_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SPH_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SPH_OK;
}

}  // namespace

extern "C" size_t sph_forces_workspace_bytes(int32_t capacity, int32_t n_cells)
{
    if (capacity < 0 || n_cells < 0) return 0;
    // per-particle equation-of-state terms (gather form), then the brick
    // counter of the persistent brick kernel
    (void)n_cells;
    return aux_bytes(capacity > 0 ? capacity : 1) + 256;
}

namespace {

// sph_forces, and with K.d_dt set sph_forces_corrector (forces may then be null)
sph_status forces_impl(const sph_grid *grid, const sph_params *params, const sph_particles *parts,
                       const uint32_t *neibs, const uint32_t *neib_count, int32_t max_neibs,
                       const int32_t *cell_start, const int32_t *cell_end, const uint16_t *neibs_brick,
                       float *forces, void *workspace, size_t workspace_bytes, void *stream, const Corrector &K)
{
    if (!common_args(grid, params, parts, neibs, neib_count, max_neibs)) return SPH_ERR_ARG;
    if (parts->n > 0 && !forces && !K.d_dt) return SPH_ERR_ARG;
    ForceConst C;
    if (!make_const(grid, params, max_neibs, C)) return SPH_ERR_ARG;
    const int shape = brick_shape_index(grid->brick);
    if (shape < 0) return SPH_ERR_ARG;
    const int64_t n_cells = (int64_t)grid->ncell[0] * grid->ncell[1] * grid->ncell[2];
    if (n_cells <= 0 || n_cells > INT32_MAX - 1) return SPH_ERR_ARG;
    if (!workspace || workspace_bytes < sph_forces_workspace_bytes(parts->capacity, (int32_t)n_cells))
        return SPH_ERR_WORKSPACE;
    const int n = parts->n;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        // the corrector's clock still advances, as the separate stage's does
        if (K.d_dt && K.d_time)
            k_add_time<<<1, 256, 0, s>>>(K.d_time, K.d_dt, K.cell_scene ? K.n_scenes : 1);
        SPH_CHECK_LAUNCH();
        return SPH_OK;
    }
    float2 *aux = (float2 *)workspace;
    int32_t *next = (int32_t *)((char *)workspace + aux_bytes(parts->capacity > 0 ? parts->capacity : 1));
    if (grid->cell_alpha && !parts->cell) return SPH_ERR_ARG;
    const bool bricks = cell_start && cell_end && neibs_brick;
    if (bricks && !parts->cell) return SPH_ERR_ARG;
    if (bricks && ((uintptr_t)neibs_brick & 15u)) return SPH_ERR_ARG;  // read in 16-byte groups
    if ((params->delta != 0.0f) && !parts->info) return SPH_ERR_ARG;
    if (bricks)
        k_zero_one<int32_t><<<1, 1, 0, s>>>(next);
    else
        k_eos<<<sph_blocks(n, kThreads), kThreads, 0, s>>>(n, (const float4 *)parts->vel, aux, parts->cell, C);
    ForceArgs a;
    a.grid = grid;
    a.shape = shape;
    a.n = n;
    a.pos = (const float4 *)parts->pos;
    a.vel = (const float4 *)parts->vel;
    a.aux = aux;
    a.cell = parts->cell;
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
    a.out = (float4 *)forces;
    a.bricks = bricks;
    a.K = K;
    static bool (*const pairs[4])(int, const ForceArgs &, const ForceConst &, hipStream_t) = {
        forces_pairs_kernel0, forces_pairs_kernel1, forces_pairs_kernel2, forces_pairs_kernel3};
    const int model = model_of(params);
    if (!pairs[model_kernel(model)](model, a, C, s)) return SPH_ERR_ARG;
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

}  // namespace

extern "C" sph_status sph_forces(const sph_grid *grid, const sph_params *params, const sph_particles *parts,
                                 const uint32_t *neibs, const uint32_t *neib_count, int32_t max_neibs,
                                 const int32_t *cell_start, const int32_t *cell_end,
                                 const uint16_t *neibs_brick, float *forces, void *workspace,
                                 size_t workspace_bytes, void *stream)
{
    const Corrector none = {};
    return forces_impl(grid, params, parts, neibs, neib_count, max_neibs, cell_start, cell_end, neibs_brick, forces,
                       workspace, workspace_bytes, stream, none);
}

extern "C" sph_status sph_forces_corrector(const sph_grid *grid, const sph_params *params,
                                           const sph_particles *star, const uint32_t *neibs,
                                           const uint32_t *neib_count, int32_t max_neibs,
                                           const int32_t *cell_start, const int32_t *cell_end,
                                           const uint16_t *neibs_brick, const double *d_dt,
                                           sph_particles *state_n, double *d_time, float *forces,
                                           void *workspace, size_t workspace_bytes, void *stream)
{
    if (!star || !state_n || !d_dt) return SPH_ERR_ARG;
    if (state_n->n != star->n || state_n->capacity < star->n) return SPH_ERR_ARG;
    if (star->n > 0) {
        if (!state_n->pos || !state_n->vel || !state_n->cell || !state_n->info) return SPH_ERR_ARG;
        // state n is rewritten while the kernel still reads state * of other
        // particles: the two must not share storage
        if (state_n->pos == star->pos || state_n->vel == star->vel) return SPH_ERR_ARG;
    }
    Corrector K = {};
    K.d_dt = d_dt;
    K.pos = (float4 *)state_n->pos;
    K.vel = (float4 *)state_n->vel;
    K.cell = state_n->cell;
    K.info = state_n->info;
    K.d_time = d_time;
    K.gx = params ? params->g[0] : 0.0f;
    K.gy = params ? params->g[1] : 0.0f;
    K.gz = params ? params->g[2] : 0.0f;
    return forces_impl(grid, params, star, neibs, neib_count, max_neibs, cell_start, cell_end, neibs_brick, forces,
                       workspace, workspace_bytes, stream, K);
}

extern "C" sph_status sph_forces_corrector_scenes(const sph_grid *grid, const sph_params *params,
                                                  const sph_particles *star, const uint32_t *neibs,
                                                  const uint32_t *neib_count, int32_t max_neibs,
                                                  const int32_t *cell_start, const int32_t *cell_end,
                                                  const uint16_t *neibs_brick, const double *d_dt,
                                                  const int32_t *cell_scene, int32_t n_scenes,
                                                  sph_particles *state_n, double *d_time, float *forces,
                                                  void *workspace, size_t workspace_bytes, void *stream)
{
    if (!star || !state_n || !d_dt || !grid || !cell_scene || n_scenes < 1 || n_scenes > SPH_MAX_SCENES)
        return SPH_ERR_ARG;
    if (state_n->n != star->n || state_n->capacity < star->n) return SPH_ERR_ARG;
    if (star->n > 0) {
        if (!state_n->pos || !state_n->vel || !state_n->cell || !state_n->info) return SPH_ERR_ARG;
        if (state_n->pos == star->pos || state_n->vel == star->vel) return SPH_ERR_ARG;
    }
    Corrector K = {};
    K.d_dt = d_dt;
    K.pos = (float4 *)state_n->pos;
    K.vel = (float4 *)state_n->vel;
    K.cell = state_n->cell;
    K.info = state_n->info;
    K.d_time = d_time;
    K.gx = params ? params->g[0] : 0.0f;
    K.gy = params ? params->g[1] : 0.0f;
    K.gz = params ? params->g[2] : 0.0f;
    K.cell_scene = cell_scene;
    K.cell_base = grid->cell_base;
    K.n_scenes = n_scenes;
    return forces_impl(grid, params, star, neibs, neib_count, max_neibs, cell_start, cell_end, neibs_brick, forces,
                       workspace, workspace_bytes, stream, K);
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

extern "C" sph_status sph_count_missed_pairs(const sph_grid *grid, const sph_params *params,
                                             const sph_particles *parts, const uint32_t *neibs,
                                             const uint32_t *neib_count, int32_t max_neibs, int32_t phase,
                                             long long *d_missed, void *stream)
{
    if (!common_args(grid, params, parts, neibs, neib_count, max_neibs) || !d_missed) return SPH_ERR_ARG;
    if (phase != 0 && phase != 1) return SPH_ERR_ARG;
    ForceConst C;
    if (!make_const(grid, params, max_neibs, C)) return SPH_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    // phase 0 counts into slot 0, phase 1 into slot 1 (both non-negative
    // counts, accumulated as unsigned)
    unsigned long long *slot = (unsigned long long *)(d_missed + phase);
    k_zero_u64<<<1, 1, 0, s>>>(slot);
    SPH_CHECK_LAUNCH();
    const int n = parts->n;
    if (n > 0)
        k_count_interactions<<<sph_blocks(n, kThreads), kThreads, 0, s>>>(n, (const float4 *)parts->pos, neibs,
                                                                          neib_count, C, slot);
    if (phase == 1) k_missed_finish<<<1, 1, 0, s>>>(d_missed);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

extern "C" sph_status sph_forces_noalloc(const sph_grid *grid, const sph_params *params,
                                         const sph_particles *parts, const uint32_t *neibs,
                                         const uint32_t *neib_count, int32_t max_neibs, const int32_t *cell_start,
                                         const int32_t *cell_end, const uint16_t *neibs_brick, float *forces,
                                         void *stream)
{
    if (!grid || !params || !parts) return SPH_ERR_ARG;
    if (parts->capacity < 0 || parts->capacity > SPH_MAX_CAPACITY) return SPH_ERR_ARG;
    const int64_t n_cells = (int64_t)grid->ncell[0] * grid->ncell[1] * grid->ncell[2];
    if (n_cells <= 0 || n_cells > INT32_MAX - 1) return SPH_ERR_ARG;
    // the size check comes before any device call
    if (sph_forces_workspace_bytes(parts->capacity, (int32_t)n_cells) > (size_t)SPH_NOALLOC_SCRATCH_BYTES)
        return SPH_ERR_SCRATCH;
    void *ws = nullptr;
    const sph_status st = noalloc_scratch(&ws);
    if (st != SPH_OK) return st;
    return sph_forces(grid, params, parts, neibs, neib_count, max_neibs, cell_start, cell_end, neibs_brick, forces,
                      ws, (size_t)SPH_NOALLOC_SCRATCH_BYTES, stream);
}
