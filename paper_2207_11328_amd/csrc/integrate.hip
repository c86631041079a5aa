// Explicit midpoint predictor/corrector and the device-side adaptive time
// step (arXiv:2207.11328, section "Code structure": predictor and corrector
// phases with dt/2 and dt; section "The GPU in GPUSPH": dt from a device
// reduction, kept on the device here so a whole step can be enqueued with
// no host round trip).
#include <hip/hip_runtime.h>
#include <math.h>

#include "sph_device.h"

using namespace sph;

namespace {

constexpr int kThreads = 256;
constexpr int kDtBlocks = 1024;

__global__ __launch_bounds__(kThreads) void k_integrate(int n, int stage, const double *__restrict__ d_dt,
                                                        const int32_t *__restrict__ cell,
                                                        const uint32_t *__restrict__ info,
                                                        const float4 *pos_n, const float4 *vel_n,
                                                        const float4 *__restrict__ vel_star,
                                                        const float4 *__restrict__ forces, float4 *pos_out,
                                                        float4 *vel_out, float gx, float gy, float gz,
                                                        double *__restrict__ d_time)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    const double dt = *d_dt;
    if (stage == 1 && d_time && i == 0) *d_time += dt;
    if (i >= n) return;
    const float tau = (float)(stage == 0 ? 0.5 * dt : dt);
    float4 p = pos_n[i];
    float4 v = vel_n[i];
    if (cell[i] >= 0) {
        const bool boundary = ptype(info[i]) == kBoundary;
        const float4 ua = stage == 0 || boundary ? v : vel_star[i];
        midpoint_stage(p, v, ua, forces[i], boundary, tau, gx, gy, gz);
    }
    pos_out[i] = p;
    vel_out[i] = v;
}

// Per-block maxima of the sound speed and of |a + g| over fluid particles.
__global__ __launch_bounds__(kThreads) void k_dt_partial(int n, const int32_t *__restrict__ cell,
                                                         const uint32_t *__restrict__ info,
                                                         const float4 *__restrict__ vel,
                                                         const float4 *__restrict__ forces, float rho0,
                                                         float inv_rho0, float c0, float gx, float gy, float gz,
                                                         float2 *__restrict__ partial)
{
    float cmax = 0.0f, amax = 0.0f;
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        if (cell[i] < 0 || ptype(info[i]) == kBoundary) continue;
        const float4 f = forces[i];
        float c, a;
        dt_speeds(vel[i].w, f.x, f.y, f.z, rho0, inv_rho0, c0, gx, gy, gz, c, a);
        cmax = fmaxf(cmax, c);
        amax = fmaxf(amax, a);
    }
    cmax = wave_max(cmax);
    amax = wave_max(amax);
    __shared__ float2 w[kThreads / kWave];
    if (threadIdx.x % kWave == 0) w[threadIdx.x / kWave] = make_float2(cmax, amax);
    __syncthreads();
    if (threadIdx.x == 0) {
        float2 r = w[0];
        for (int k = 1; k < kThreads / kWave; ++k) {
            r.x = fmaxf(r.x, w[k].x);
            r.y = fmaxf(r.y, w[k].y);
        }
        partial[blockIdx.x] = r;
    }
}

__global__ __launch_bounds__(kThreads) void k_dt_final(int np, const float2 *__restrict__ partial, double h,
                                                       double nu, double cfl, double *__restrict__ d_dt)
{
    float cmax = 0.0f, amax = 0.0f;
    for (int k = threadIdx.x; k < np; k += kThreads) {
        cmax = fmaxf(cmax, partial[k].x);
        amax = fmaxf(amax, partial[k].y);
    }
    cmax = wave_max(cmax);
    amax = wave_max(amax);
    __shared__ float2 w[kThreads / kWave];
    if (threadIdx.x % kWave == 0) w[threadIdx.x / kWave] = make_float2(cmax, amax);
    __syncthreads();
    if (threadIdx.x == 0) {
        double c = 0.0, a = 0.0;
        for (int k = 0; k < kThreads / kWave; ++k) {
            c = fmax(c, (double)w[k].x);
            a = fmax(a, (double)w[k].y);
        }
        *d_dt = dt_from_maxima(c, a, h, nu, cfl);
    }
}

// Reverse of the midpoint stages (the transpose of the linear updates).
//   stage 1:  gpos/gvel hold dL/dy^{n+1}; they stay as the direct part of
//             dL/dy^n.  Writes the upstream of the derivatives at y*
//             gforce = (dt dL/du^{n+1} (fluid), dt dL/drho^{n+1}) and initialises
//             dL/dy* = (0, dt dL/do^{n+1} (fluid), 0) in gpos_s/gvel_s.
//   stage 0:  gpos_s/gvel_s hold the complete dL/dy*.  Adds it to dL/dy^n
//             (plus tau dL/do* to the fluid velocity) and writes the upstream
//             of the derivatives at y^n: gforce = (tau dL/du* (fluid), tau dL/drho*).
__global__ __launch_bounds__(kThreads) void k_integrate_backward(int n, int stage, const double *__restrict__ d_dt,
                                                                 const int32_t *__restrict__ cell,
                                                                 const uint32_t *__restrict__ info,
                                                                 float4 *__restrict__ gpos, float4 *__restrict__ gvel,
                                                                 float4 *__restrict__ gpos_s,
                                                                 float4 *__restrict__ gvel_s,
                                                                 float4 *__restrict__ gforce)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const double dt = *d_dt;
    const bool valid = cell[i] >= 0;
    const bool fluid = valid && ptype(info[i]) != kBoundary;
    if (stage == 1) {
        const float t = (float)dt;
        const float4 go = gpos[i], gv = gvel[i];
        gforce[i] = make_float4(fluid ? t * gv.x : 0.0f, fluid ? t * gv.y : 0.0f, fluid ? t * gv.z : 0.0f,
                                valid ? t * gv.w : 0.0f);
        gpos_s[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        gvel_s[i] = make_float4(fluid ? t * go.x : 0.0f, fluid ? t * go.y : 0.0f, fluid ? t * go.z : 0.0f, 0.0f);
    } else {
        const float tau = (float)(0.5 * dt);
        const float4 so = gpos_s[i], sv = gvel_s[i];
        float4 go = gpos[i], gv = gvel[i];
        go.x += so.x;
        go.y += so.y;
        go.z += so.z;
        gv.x += sv.x + (fluid ? tau * so.x : 0.0f);
        gv.y += sv.y + (fluid ? tau * so.y : 0.0f);
        gv.z += sv.z + (fluid ? tau * so.z : 0.0f);
        gv.w += sv.w;
        gpos[i] = go;
        gvel[i] = gv;
        gforce[i] = make_float4(fluid ? tau * sv.x : 0.0f, fluid ? tau * sv.y : 0.0f, fluid ? tau * sv.z : 0.0f,
                                valid ? tau * sv.w : 0.0f);
    }
}

// FP64 conservation diagnostics, two-level fixed-order reduction (the
// result does not depend on scheduling).  Per particle i < n with cell >= 0:
//   [0] m   [1..3] m u (fluid)   [4..6] m a (forces xyz; all particles)
//   [7] m / rho   [8] n fluid   [9] n boundary   [10] max |rho/rho0 - 1| (fluid)
//   [11] 1/2 m |u|^2 (fluid)
constexpr int kDiag = 12;
constexpr int kDiagBlocks = 1024;

__global__ __launch_bounds__(kThreads) void k_diag_partial(int n, const int32_t *__restrict__ cell,
                                                           const uint32_t *__restrict__ info,
                                                           const float4 *__restrict__ pos,
                                                           const float4 *__restrict__ vel,
                                                           const float4 *__restrict__ forces, float rho0,
                                                           double *__restrict__ partial)
{
    double acc[kDiag];
#pragma unroll
    for (int k = 0; k < kDiag; ++k) acc[k] = 0.0;
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        if (cell[i] < 0) continue;
        const float4 p = pos[i], v = vel[i];
        const double m = p.w;
        const bool fluid = ptype(info[i]) != kBoundary;
        acc[0] += m;
        if (fluid) {
            acc[1] += m * v.x;
            acc[2] += m * v.y;
            acc[3] += m * v.z;
            acc[8] += 1.0;
            acc[10] = fmax(acc[10], fabs((double)v.w / rho0 - 1.0));
            acc[11] += 0.5 * m * ((double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z);
        } else {
            acc[9] += 1.0;
        }
        if (forces) {
            const float4 f = forces[i];
            acc[4] += m * f.x;
            acc[5] += m * f.y;
            acc[6] += m * f.z;
        }
        acc[7] += m / (double)v.w;
    }
    __shared__ double red[kDiag][kThreads / kWave];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < kDiag; ++k) {
        const double t = k == 10 ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) red[k][w] = t;
    }
    __syncthreads();
    if (threadIdx.x < kDiag) {
        const int k = threadIdx.x;
        double t = red[k][0];
        for (int q = 1; q < kThreads / kWave; ++q) t = k == 10 ? fmax(t, red[k][q]) : t + red[k][q];
        partial[(size_t)blockIdx.x * kDiag + k] = t;
    }
}

__global__ __launch_bounds__(kThreads) void k_diag_final(int np, const double *__restrict__ partial,
                                                         double *__restrict__ out)
{
    // one thread per quantity, blocks in a fixed order
    if (threadIdx.x < kDiag) {
        const int k = threadIdx.x;
        double t = 0.0;
        for (int b = 0; b < np; ++b) {
            const double v = partial[(size_t)b * kDiag + k];
            t = k == 10 ? fmax(t, v) : t + v;
        }
        out[k] = t;
    }
}

}  // namespace

extern "C" size_t sph_diagnostics_workspace_bytes(void) { return sizeof(double) * kDiag * kDiagBlocks; }

extern "C" sph_status sph_reduce_diagnostics(const sph_params *params, const sph_particles *parts,
                                             const float *forces, double *d_out, void *workspace,
                                             size_t workspace_bytes, void *stream)
{
    if (!params || !parts || !d_out) return SPH_ERR_ARG;
    const int n = parts->n;
    if (n < 0 || parts->capacity < n) return SPH_ERR_ARG;
    if (n > 0 && (!parts->cell || !parts->pos || !parts->vel || !parts->info)) return SPH_ERR_ARG;
    if (!(params->rho0 > 0.0f)) return SPH_ERR_ARG;
    if (!workspace || workspace_bytes < sph_diagnostics_workspace_bytes()) return SPH_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const unsigned want = n > 0 ? sph_blocks(n, kThreads) : 1;
    const int blocks = (int)(want < (unsigned)kDiagBlocks ? want : (unsigned)kDiagBlocks);
    double *partial = (double *)workspace;
    k_diag_partial<<<blocks, kThreads, 0, s>>>(n, parts->cell, parts->info, (const float4 *)parts->pos,
                                               (const float4 *)parts->vel, (const float4 *)forces, params->rho0,
                                               partial);
    k_diag_final<<<1, 64, 0, s>>>(blocks, partial, d_out);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

extern "C" sph_status sph_integrate_backward(const sph_params *params, int32_t stage, const double *d_dt,
                                             const sph_particles *state_n, float *grad_pos, float *grad_vel,
                                             float *grad_pos_star, float *grad_vel_star, float *grad_forces,
                                             void *stream)
{
    if (!params || !d_dt || !state_n || (stage != 0 && stage != 1)) return SPH_ERR_ARG;
    const int n = state_n->n;
    if (n < 0 || state_n->capacity < n) return SPH_ERR_ARG;
    if (n == 0) return SPH_OK;
    if (!state_n->cell || !state_n->info || !grad_pos || !grad_vel || !grad_pos_star || !grad_vel_star ||
        !grad_forces)
        return SPH_ERR_ARG;
    k_integrate_backward<<<sph_blocks(n, kThreads), kThreads, 0, (hipStream_t)stream>>>(
        n, stage, d_dt, state_n->cell, state_n->info, (float4 *)grad_pos, (float4 *)grad_vel,
        (float4 *)grad_pos_star, (float4 *)grad_vel_star, (float4 *)grad_forces);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

// Scenes sharing one grid (batching): scene of a particle in cell c is
// cell_scene[c - cell_base]; particles outside the grid, and cells whose
// entry is not in [0, n_scenes), have none.

// The predictor/corrector with the step of each particle's scene; thread k <
// n_scenes of the corrector also advances scene k's clock.
__global__ __launch_bounds__(kThreads) void k_integrate_scenes(
    int n, int stage, const double *__restrict__ d_dt, const int32_t *__restrict__ cell_scene, int cell_base,
    int n_scenes, const int32_t *__restrict__ cell, const uint32_t *__restrict__ info, const float4 *pos_n,
    const float4 *vel_n, const float4 *__restrict__ vel_star, const float4 *__restrict__ forces, float4 *pos_out,
    float4 *vel_out, float gx, float gy, float gz, double *__restrict__ d_time)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (stage == 1 && d_time && i < n_scenes) d_time[i] += d_dt[i];
    if (i >= n) return;
    float4 p = pos_n[i];
    float4 v = vel_n[i];
    const int c = cell[i];
    const int sc = c >= 0 ? cell_scene[c - cell_base] : -1;
    if ((unsigned)sc < (unsigned)n_scenes) {  // (a cell of no scene: left as it is)
        const double dt = d_dt[sc];
        const float tau = (float)(stage == 0 ? 0.5 * dt : dt);
        const bool boundary = ptype(info[i]) == kBoundary;
        const float4 ua = stage == 0 || boundary ? v : vel_star[i];
        midpoint_stage(p, v, ua, forces[i], boundary, tau, gx, gy, gz);
    }
    pos_out[i] = p;
    vel_out[i] = v;
}

__global__ __launch_bounds__(kThreads) void k_zero_u32(int n, uint32_t *__restrict__ p)
{
    for (int k = blockIdx.x * kThreads + threadIdx.x; k < n; k += gridDim.x * kThreads) p[k] = 0u;
}

// Per-scene maxima of the sound speed and of |a + g| over fluid particles,
// as float32 bit patterns (non-negative floats order as their bits), in
// m[2 s] and m[2 s + 1].  A wave takes kDtChunk consecutive particles: they
// are sorted by cell, and a scene is a run of cells, so the chunk meets its
// scenes one after the other.  The lanes that share a scene are reduced
// together, the wave keeps the running maxima of its current scene, and it
// takes the device-wide maximum once per scene it leaves (a few atomics per
// chunk, spread over the scenes).  A maximum does not depend on the order of
// the updates.
constexpr int kDtChunk = 8 * kWave;
__global__ __launch_bounds__(kThreads) void k_dt_scenes_partial(
    int n, const int32_t *__restrict__ cell, const uint32_t *__restrict__ info, const float4 *__restrict__ vel,
    const float4 *__restrict__ forces, const int32_t *__restrict__ cell_scene, int cell_base, int n_scenes,
    float rho0, float inv_rho0, float c0, float gx, float gy, float gz, uint32_t *__restrict__ m)
{
    const int lane = threadIdx.x % kWave;
    const int wave = (int)((blockIdx.x * kThreads + threadIdx.x) / kWave);
    const int begin = wave * kDtChunk, end = min(begin + kDtChunk, n);
    int cur = -1;  // the wave's current scene and its running maxima (uniform)
    float cc = 0.0f, ca = 0.0f;
    for (int i0 = begin; i0 < end; i0 += kWave) {  // uniform
        const int i = i0 + lane;
        int sc = -1;
        float c = 0.0f, a = 0.0f;
        if (i < end && cell[i] >= 0 && ptype(info[i]) != kBoundary) sc = cell_scene[cell[i] - cell_base];
        if ((unsigned)sc >= (unsigned)n_scenes) sc = -1;  // a cell of no scene counts in none
        if (sc >= 0) {
            const float4 f = forces[i];
            dt_speeds(vel[i].w, f.x, f.y, f.z, rho0, inv_rho0, c0, gx, gy, gz, c, a);
            c = fmaxf(c, 0.0f);  // (NaN or negative: no bound, as in the one-scene maxima)
            a = fmaxf(a, 0.0f);
        }
        uint64_t pending = __builtin_amdgcn_ballot_w64(sc >= 0);
        while (pending) {  // uniform
            const int leader = __builtin_ffsll((long long)pending) - 1;
            const int s = __shfl(sc, leader);
            const bool mine = sc == s;
            const float cm = wave_max(mine ? c : 0.0f), am = wave_max(mine ? a : 0.0f);
            if (s != cur) {
                if (cur >= 0 && lane == 0) {
                    atomicMax(&m[2 * cur], __float_as_uint(cc));
                    atomicMax(&m[2 * cur + 1], __float_as_uint(ca));
                }
                cur = s;
                cc = cm;
                ca = am;
            } else {
                cc = fmaxf(cc, cm);
                ca = fmaxf(ca, am);
            }
            pending &= ~__builtin_amdgcn_ballot_w64(mine);
        }
    }
    if (cur >= 0 && lane == 0) {
        atomicMax(&m[2 * cur], __float_as_uint(cc));
        atomicMax(&m[2 * cur + 1], __float_as_uint(ca));
    }
}

// dt of each scene from its maxima, as k_dt_final does for one scene.
__global__ __launch_bounds__(kThreads) void k_dt_scenes_final(int n_scenes, const uint32_t *__restrict__ m,
                                                              double h, double nu, double cfl,
                                                              double *__restrict__ d_dt)
{
    const int s = blockIdx.x * kThreads + threadIdx.x;
    if (s >= n_scenes) return;
    const double c = (double)__uint_as_float(m[2 * s]), a = (double)__uint_as_float(m[2 * s + 1]);
    d_dt[s] = dt_from_maxima(c, a, h, nu, cfl);
}

extern "C" sph_status sph_integrate(const sph_params *params, int32_t stage, const double *d_dt,
                                    const sph_particles *state_n, const float *vel_star, const float *forces,
                                    sph_particles *out, double *d_time, void *stream)
{
    if (!params || !d_dt || !state_n || !out || (stage != 0 && stage != 1)) return SPH_ERR_ARG;
    const int n = state_n->n;
    if (n < 0 || state_n->capacity < n || out->capacity < n) return SPH_ERR_ARG;
    if (n > 0) {
        if (!state_n->cell || !state_n->pos || !state_n->vel || !state_n->info || !forces) return SPH_ERR_ARG;
        if (!out->pos || !out->vel) return SPH_ERR_ARG;
        if (stage == 1 && !vel_star) return SPH_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const unsigned blocks = n > 0 ? sph_blocks(n, kThreads) : 1;
    k_integrate<<<blocks, kThreads, 0, s>>>(n, stage, d_dt, state_n->cell, state_n->info,
                                            (const float4 *)state_n->pos, (const float4 *)state_n->vel,
                                            (const float4 *)vel_star, (const float4 *)forces,
                                            (float4 *)out->pos, (float4 *)out->vel, params->g[0], params->g[1],
                                            params->g[2], d_time);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

extern "C" size_t sph_dt_workspace_bytes(void) { return sizeof(float2) * kDtBlocks; }

extern "C" sph_status sph_step_dt(const sph_params *params, const sph_particles *parts, const float *forces,
                                  double *d_dt, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!params || !parts || !d_dt) return SPH_ERR_ARG;
    const int n = parts->n;
    if (n < 0 || parts->capacity < n) return SPH_ERR_ARG;
    if (n > 0 && (!parts->cell || !parts->vel || !parts->info || !forces)) return SPH_ERR_ARG;
    if (!(params->h > 0.0f) || !(params->rho0 > 0.0f) || params->gamma != 7.0f) return SPH_ERR_ARG;
    if (!workspace || workspace_bytes < sph_dt_workspace_bytes()) return SPH_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const unsigned want = n > 0 ? sph_blocks(n, kThreads) : 1;
    const int blocks = (int)(want < (unsigned)kDtBlocks ? want : (unsigned)kDtBlocks);
    float2 *partial = (float2 *)workspace;
    k_dt_partial<<<blocks, kThreads, 0, s>>>(n, parts->cell, parts->info, (const float4 *)parts->vel,
                                             (const float4 *)forces, params->rho0,
                                             (float)(1.0 / (double)params->rho0), params->c0, params->g[0],
                                             params->g[1], params->g[2], partial);
    k_dt_final<<<1, kThreads, 0, s>>>(blocks, partial, params->h, params->nu, params->cfl, d_dt);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

extern "C" size_t sph_dt_scenes_workspace_bytes(int32_t n_scenes)
{
    if (n_scenes < 1 || n_scenes > SPH_MAX_SCENES) return 0;
    return (size_t)(2 * sizeof(uint32_t) * (size_t)n_scenes + 256);
}

static bool scene_table_ok(const sph_grid *grid, const int32_t *cell_scene, int32_t n_scenes)
{
    if (!grid || !cell_scene || n_scenes < 1 || n_scenes > SPH_MAX_SCENES) return false;
    const int64_t n_cells = (int64_t)grid->ncell[0] * grid->ncell[1] * grid->ncell[2];
    return n_cells > 0 && n_cells <= INT32_MAX;
}

extern "C" sph_status sph_step_dt_scenes(const sph_grid *grid, const sph_params *params,
                                         const sph_particles *parts, const float *forces,
                                         const int32_t *cell_scene, int32_t n_scenes, double *d_dt,
                                         void *workspace, size_t workspace_bytes, void *stream)
{
    if (!params || !parts || !d_dt || !scene_table_ok(grid, cell_scene, n_scenes)) return SPH_ERR_ARG;
    const int n = parts->n;
    if (n < 0 || parts->capacity < n) return SPH_ERR_ARG;
    if (n > 0 && (!parts->cell || !parts->vel || !parts->info || !forces)) return SPH_ERR_ARG;
    if (!(params->h > 0.0f) || !(params->rho0 > 0.0f) || params->gamma != 7.0f) return SPH_ERR_ARG;
    if (!workspace || workspace_bytes < sph_dt_scenes_workspace_bytes(n_scenes)) return SPH_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    uint32_t *m = (uint32_t *)workspace;
    const unsigned zb = sph_blocks(2 * n_scenes, kThreads);
    k_zero_u32<<<zb, kThreads, 0, s>>>(2 * n_scenes, m);
    if (n > 0) {
        const int waves = (n + kDtChunk - 1) / kDtChunk;
        const unsigned blocks = sph_blocks(waves * kWave, kThreads);
        k_dt_scenes_partial<<<blocks, kThreads, 0, s>>>(n, parts->cell, parts->info, (const float4 *)parts->vel,
                                                         (const float4 *)forces, cell_scene, grid->cell_base,
                                                         n_scenes, params->rho0, (float)(1.0 / (double)params->rho0),
                                                         params->c0, params->g[0], params->g[1], params->g[2], m);
    }
    k_dt_scenes_final<<<sph_blocks(n_scenes, kThreads), kThreads, 0, s>>>(n_scenes, m, params->h, params->nu,
                                                                          params->cfl, d_dt);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

extern "C" sph_status sph_integrate_scenes(const sph_grid *grid, const sph_params *params, int32_t stage,
                                           const double *d_dt, const int32_t *cell_scene, int32_t n_scenes,
                                           const sph_particles *state_n, const float *vel_star,
                                           const float *forces, sph_particles *out, double *d_time, void *stream)
{
    if (!params || !d_dt || !state_n || !out || (stage != 0 && stage != 1)) return SPH_ERR_ARG;
    if (!scene_table_ok(grid, cell_scene, n_scenes)) return SPH_ERR_ARG;
    const int n = state_n->n;
    if (n < 0 || state_n->capacity < n || out->capacity < n) return SPH_ERR_ARG;
    if (n > 0) {
        if (!state_n->cell || !state_n->pos || !state_n->vel || !state_n->info || !forces) return SPH_ERR_ARG;
        if (!out->pos || !out->vel) return SPH_ERR_ARG;
        if (stage == 1 && !vel_star) return SPH_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const int threads = n > n_scenes ? n : n_scenes;
    k_integrate_scenes<<<sph_blocks(threads, kThreads), kThreads, 0, s>>>(
        n, stage, d_dt, cell_scene, grid->cell_base, n_scenes, state_n->cell, state_n->info,
        (const float4 *)state_n->pos, (const float4 *)state_n->vel, (const float4 *)vel_star,
        (const float4 *)forces, (float4 *)out->pos, (float4 *)out->vel, params->g[0], params->g[1], params->g[2],
        d_time);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}

extern "C" const char *sph_status_string(sph_status st)
{
    switch (st) {
    case SPH_OK: return "SPH_OK";
    case SPH_ERR_ARG: return "SPH_ERR_ARG: invalid argument or shape";
    case SPH_ERR_WORKSPACE: return "SPH_ERR_WORKSPACE: workspace missing or too small";
    case SPH_ERR_HIP: return "SPH_ERR_HIP: HIP launch or runtime failure";
    case SPH_ERR_SCRATCH:
        return "SPH_ERR_SCRATCH: the problem needs more than the fixed device scratch of sph_forces_noalloc "
               "(SPH_NOALLOC_SCRATCH_BYTES)";
    }
    return "SPH: unknown status";
}

extern "C" int32_t sph_abi_version(void) { return 3; }
