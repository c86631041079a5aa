/*
 * sph.h — C ABI of the MI355X weakly-compressible SPH step library (libsph.so).
 *
 * The library implements the step that dominates a WCSPH run, as stated in
 * arXiv:2207.11328 (section "From theory to implementation"): a neighbour
 * search (re-bin, sort by cell, cell ranges, per-particle neighbour list), the
 * time derivatives ("forces": continuity, Cole equation of state, golden-rule
 * or Landrini-Morris pressure gradient plus artificial and optional laminar
 * viscosity, density diffusion, Wendland, cubic-spline, quadratic or Gaussian
 * kernel) and a predictor/corrector integrator; plus the adjoint of the
 * derivatives.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All particle arrays, lists and scalars marked "device" are device
 *   pointers on the current HIP device; the caller allocates and owns them.
 *   The library never allocates on these paths and keeps no state between
 *   calls except the compute-unit count of each device it has run on (queried
 *   once; it sizes the grids of the persistent brick kernels).
 * - `stream` is a hipStream_t passed as void*; NULL means the default
 *   stream.  Every call only enqueues work on that stream (asynchronous);
 *   calls on distinct streams with distinct buffers may overlap.
 * - Argument and shape errors are reported synchronously by the return code
 *   and nothing is launched.  Conditions discovered on the device (neighbour
 *   overflow, particles leaving the grid) are written to a device status
 *   word and are visible after the caller synchronises the stream.  No call
 *   aborts or throws.
 * - Particle state is structure-of-arrays (section "From theory to
 *   implementation"): positions are cell-relative (section "Optimizing the
 *   neighbors search"): a linear cell index plus a float32 offset from the
 *   cell centre, so float32 keeps uniform accuracy over large domains.
 *     cell[i]  int32  cx + ncell[0]*(cy + ncell[1]*cz) + cell_base; -1 after
 *                     a build for a particle that left the grid
 *     pos[i]   float4 xyz: offset from the cell centre [m], w: mass [kg]
 *     vel[i]   float4 xyz: velocity [m/s], w: density [kg/m^3]
 *     info[i]  uint32 type << 30 | id; type 0 = fluid, 1 = fixed ("dynamic")
 *                     boundary particle; ids unique
 * - After sph_build_neighbors the particles are stored sorted by
 *   (cell, type, id), and neighbour indices refer to that order.
 *
 * Neighbour list (sections "Efficient split neighbors list" and
 * "Changing perspective: from the particle to the cell")
 * -----------------------------------------------------
 * Fixed size, `max_neibs` slots per particle, neighbour-major inside tiles of
 * 64 particles (one wave64):
 *     slot k of particle i is neibs[(i / 64) * (64 * max_neibs) + 64 * k + i % 64]
 * so slot k of 64 consecutive particles is one contiguous 256-byte row and
 * every offset inside a tile fits 32 bits.  The array holds
 * sph_neib_list_entries(capacity, max_neibs) entries.  Fluid neighbours fill slots
 * 0, 1, ... upwards, boundary neighbours fill max_neibs-1, max_neibs-2, ...
 * downwards.  neib_count[i] = n_fluid | n_boundary << 16 replaces the paper's
 * end-of-list marker.  A boundary particle lists fluid neighbours only.  Each
 * entry packs the neighbour's sorted index j (bits 0..25, so capacity is at
 * most 2^26) and the cell difference k_d = c_i,d - c_j,d in {-1, 0, 1} of
 * each axis d as a two's-complement 2-bit field (bits 26+2d .. 27+2d),
 * periodic images already resolved.  The separation is then
 * x_ij = k * cell_size + (o_i - o_j).
 *
 * A pair is listed iff, in float32 with every operation rounded,
 *   x_d = (k_d * cs_d) + (o_i,d - o_j,d),   r2 = (x*x + y*y) + z*z,
 *   r2 < r_search * r_search.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPH_OK = 0,
    SPH_ERR_ARG = 1,        /* invalid argument or shape; nothing launched */
    SPH_ERR_WORKSPACE = 2,  /* workspace missing or smaller than required */
    SPH_ERR_HIP = 3,        /* a HIP runtime call or launch failed */
    SPH_ERR_SCRATCH = 4     /* the problem needs more device scratch than the
                               fixed maximum of sph_forces_noalloc */
} sph_status;

/* Device status word written by sph_build_neighbors: int32[SPH_STATUS_WORDS]. */
enum {
    SPH_STATUS_N_ACTIVE = 0,   /* particles inside the grid (sorted first)  */
    SPH_STATUS_MAX_NEIBS = 1,  /* largest n_fluid + n_boundary found        */
    SPH_STATUS_OVERFLOW = 2,   /* particles whose list did not fit          */
    SPH_STATUS_DROPPED = 3,    /* particles that left the grid (sorted last) */
    SPH_STATUS_NONFINITE = 4,  /* particles with a non-finite offset, mass,
                                  velocity or density when the build ran    */
    SPH_STATUS_WORDS = 8       /* words 5..7 are reserved and written 0     */
};

#define SPH_NEIB_INDEX_BITS 26
#define SPH_MAX_CAPACITY (1 << SPH_NEIB_INDEX_BITS)

/* Uniform cell grid (section "Optimizing the neighbors search"): origin,
 * extents and spacing.  cell_size[d] must be >= r_search; a periodic axis
 * (bit d of `periodic`) has ncell[d] >= 3 and period ncell[d] * cell_size[d].
 * Several independent scenes can share one grid (one neighbour search, one
 * launch per step for all of them): place them in disjoint regions separated
 * by at least one empty cell layer, so no pair across scenes is ever listed,
 * and give each region its own artificial-viscosity coefficient through
 * cell_alpha (device float[n_cells], indexed by cell - cell_base; NULL means
 * params->alpha everywhere; the coefficient of a pair is that of the central
 * particle's cell, equal for both members within one scene).
 * brick: cells per brick along x, y, z of the LDS kernels (list build,
 * sph_forces, sph_forces_backward), one of sph_brick_shapes; {0, 0, 0} is
 * the default shape.  Lists built with one shape are read with the same. */
typedef struct {
    double origin[3];
    float cell_size[3];
    int32_t ncell[3];
    uint32_t periodic;
    int32_t cell_base;
    const float *cell_alpha;
    int32_t brick[3];
} sph_grid;

/* Smoothing kernels (listing l:ktemplate), all of support 2h, q = r/h,
 * normalised to unit integral in 3D, F = (1/r) dW/dr:
 *   SPH_KERNEL_WENDLAND      W = 21/(16 pi h^3) (1 - q/2)^4 (2q + 1)
 *   SPH_KERNEL_CUBIC_SPLINE  W = 1/(pi h^3) (1 - 3/2 q^2 + 3/4 q^3) for q < 1,
 *                                1/(4 pi h^3) (2 - q)^3 for 1 <= q < 2
 *   SPH_KERNEL_QUADRATIC     W = 15/(64 pi h^3) (2 - q)^2 (pairs at r = 0,
 *                                where its F is unbounded, contribute nothing)
 *   SPH_KERNEL_GAUSSIAN      W = C (exp(-q^2) - exp(-4)), the Gaussian
 *                                truncated at d = 2h, 1/C = 4 pi h^3
 *                                (sqrt(pi)/4 erf(2) - 11/3 exp(-4)) */
enum { SPH_KERNEL_WENDLAND = 0, SPH_KERNEL_CUBIC_SPLINE = 1, SPH_KERNEL_QUADRATIC = 2, SPH_KERNEL_GAUSSIAN = 3 };

/* Laminar viscosity term (section "Minimizing complexity"), added to the
 * artificial viscosity: none, Morris, or Monaghan's K form with K = 5. */
enum { SPH_VISC_ARTIFICIAL = 0, SPH_VISC_MORRIS = 1, SPH_VISC_MONAGHAN_K = 2 };

/* Formulation of the continuity and momentum sums. */
enum { SPH_FORM_GOLDEN_RULE = 0, SPH_FORM_LANDRINI_MORRIS = 1 };

/* Physical and numerical parameters.
 *   h          smoothing length; every kernel has support 2h
 *   r_search   neighbour search radius (>= 2h; the excess is the skin that
 *              lets the list be reused for several steps)
 *   rho0, gamma, c0   Cole equation of state P = B((rho/rho0)^gamma - 1),
 *              B = rho0 c0^2 / gamma (gamma = 7 only)
 *   alpha, eps_visc   Monaghan artificial viscosity
 *              Pi_ij = -alpha h cbar (u_ij.x_ij) / (rhobar (r^2 + eps h^2))
 *              for approaching pairs, cbar and rhobar arithmetic means
 *              (always applied; alpha = 0 disables it)
 *   nu, visc_model   kinematic viscosity and laminar term, weight
 *              m_j/(rho_i rho_j) and mu_bar the harmonic mean of rho nu:
 *              SPH_VISC_MORRIS:     sum_j 4 nu m_j / (rho_i + rho_j) F_ij u_ij
 *              SPH_VISC_MONAGHAN_K: K sum_j 4 nu m_j / (rho_i + rho_j) F_ij
 *                                   (u_ij.x_ij) / (r^2 + eps h^2) x_ij, K = 5
 *                                   (d + 2: the term tends to nu lap u for
 *                                   a divergence-free flow)
 *              SPH_VISC_ARTIFICIAL: no laminar term
 *   g          body acceleration added to fluid particles by the integrator
 *   cfl        time-step safety factor
 *   delta      density diffusion of Molteni and Colagrossi (the mass
 *              dissipative term named in section "A lightning introduction
 *              to the method", used by the paper's test cases), between
 *              fluid particles only:
 *              Drho_i/Dt += -2 delta h c0 sum_j (rho_j - rho_i) F_ij r^2 /
 *                           (r^2 + eps h^2) m_j / rho_j;  0 disables it
 *   kernel     SPH_KERNEL_* (0, Wendland, for a zero-initialised struct)
 *   formulation  SPH_FORM_GOLDEN_RULE (eq. mass-cont-sph1, eq. ns-sph1) or
 *              SPH_FORM_LANDRINI_MORRIS (eq. mass-cont-sph2, eq. ns-sph2) */
typedef struct {
    float h, r_search, rho0, gamma, c0, alpha, eps_visc, nu;
    float g[3];
    float cfl;
    int32_t visc_model;
    float delta;
    int32_t kernel;
    int32_t formulation;
} sph_params;

/* Particle arrays (device pointers), see the conventions above. */
typedef struct {
    int32_t n;          /* particles stored */
    int32_t capacity;   /* allocated length of every per-particle array */
    int32_t *cell;
    float *pos;         /* [capacity][4] */
    float *vel;         /* [capacity][4] */
    uint32_t *info;
} sph_particles;

/* Human-readable name of a status code (static storage). */
const char *sph_status_string(sph_status s);

/* ABI revision of this header (incremented on incompatible changes; 2: the
 * status word grew to SPH_STATUS_WORDS; 3: per-scene time steps). */
int32_t sph_abi_version(void);

/* Number of uint32 entries of a neighbour list for `capacity` particles:
 * ceil(capacity / 64) * 64 * max_neibs. */
size_t sph_neib_list_entries(int32_t capacity, int32_t max_neibs);

/* Entries (uint16) of a brick-local neighbour list for `capacity`
 * particles: ceil(capacity / 64) * 64 * 8 * ceil(max_neibs / 8) list
 * entries, then the table of the bricks with a pair (capacity + 4 int32
 * words, i.e. 2 * (capacity + 4) entries; see sph_build_neighbors). */
size_t sph_neib_brick_entries(int32_t capacity, int32_t max_neibs);

/* Brick shapes the LDS kernels support: writes up to max_shapes triples
 * (cells along x, y, z; host memory shapes[3 * max_shapes], may be NULL) and
 * returns how many there are.  The first is the default.  Bricks tile the
 * grid from cell 0 along each axis; a workgroup of the list build and of
 * the derivative kernels owns one brick. */
int32_t sph_brick_shapes(int32_t *shapes, int32_t max_shapes);

/* Bytes of device workspace sph_build_neighbors needs. */
size_t sph_build_workspace_bytes(int32_t capacity, int32_t n_cells);

/* Neighbour search (sections "Optimizing the neighbors search", "Efficient
 * split neighbors list", "Changing perspective: from the particle to the
 * cell"): in one call on `stream`,
 *   1. re-bin: offsets that drifted out of [-cs/2, cs/2) move by whole cells
 *      (at most 4 per axis, float32, periodic axes wrap); particles leaving
 *      the grid or with non-finite offsets get cell = -1;
 *   2. sort particles by (cell, type, id), dropped ones last, and reorder
 *      cell/pos/vel/info in place (parts is in/out; parts->n is unchanged);
 *   3. cell ranges: particles of linear cell c (relative to cell_base) are
 *      [cell_start[c], cell_end[c]) (device int32[n_cells] each);
 *   4. build the split neighbour list described above into
 *      neibs (device uint32[sph_neib_list_entries(capacity, max_neibs)]) and
 *      neib_count (device uint32[capacity]); dropped particles get count 0;
 *   5. d_status (device int32[SPH_STATUS_WORDS], see SPH_STATUS_*) is
 *      overwritten; a particle whose offset, mass, velocity or density is
 *      not finite is counted in SPH_STATUS_NONFINITE (a non-finite offset
 *      also drops it), so that a state that blew up is reported at the next
 *      rebuild instead of propagating silently;
 *   6. if perm_out (device uint32[capacity]) is not NULL, perm_out[k] is the
 *      index before the call of the particle now stored at k (k < n); the
 *      adjoint of the rebuild is dL/dy_before[perm_out[k]] = dL/dy_after[k]
 *      (sph_unpermute), since re-binning does not move a particle;
 *   7. if neibs_brick (device uint16[sph_neib_brick_entries(capacity,
 *      max_neibs)], 16-byte aligned: it is written and read in 16-byte
 *      groups; SPH_ERR_ARG otherwise) is not NULL, the same lists in brick-local form for
 *      sph_forces: entry k of particle i (k < nf + nb, neighbours in scan
 *      order, fluid and boundary interleaved as found) is stored at
 *        ((i / 64) * G + k / 8) * 512 + (i % 64) * 8 + k % 8,
 *      G = ceil(max_neibs / 8) (groups of 8 entries, one 16-byte load per
 *      particle and group), and holds the neighbour's position in the staging
 *      order of the brick
 *      (grid->brick) that holds i; staging order: the cells of the brick
 *      and its one-cell halo, x fastest, then z, then y, periodic axes
 *      wrapped, cells outside a closed axis empty, then particles of a cell
 *      in sorted order;
 *      saturated at 65535.  Behind the lists (at entry ceil(capacity / 64)
 *      * 64 * 8 * ceil(max_neibs / 8), as int32 words) the table of the
 *      bricks that hold a particle with a non-empty list, for the brick
 *      form of sph_forces: [0] the number of heavy bricks (at least 12
 *      particles per inner cell), [1 .. capacity] brick ids bx + nbx (by +
 *      nby bz) of the grid tiled by grid->brick from cell 0, the heavy ones
 *      from the front and the light ones from the back, [capacity + 1] the
 *      number of light bricks, [capacity + 2 ..] reserved (capacity is at
 *      least 1 here);
 * A particle whose neighbours exceed max_neibs keeps the first max_neibs
 * found (scan order: cells z, y, x outer to inner, then sorted index) and is
 * counted in SPH_STATUS_OVERFLOW; the lists are then unusable for physics.
 * workspace: device buffer of at least sph_build_workspace_bytes bytes.
 * Errors: SPH_ERR_ARG for null pointers, n > capacity, capacity > 2^26,
 * max_neibs outside [1, 65535], bad grid or brick shape; SPH_ERR_WORKSPACE. */
sph_status sph_build_neighbors(const sph_grid *grid, const sph_params *params,
                               sph_particles *parts, uint32_t *neibs, uint32_t *neib_count,
                               int32_t max_neibs, int32_t *cell_start, int32_t *cell_end,
                               int32_t *d_status, uint32_t *perm_out, uint16_t *neibs_brick,
                               void *workspace, size_t workspace_bytes, void *stream);

/* Time derivatives (eq. mass-cont-sph1 and eq. ns-sph1 with the readings of
 * the design notes, or eq. mass-cont-sph2 and eq. ns-sph2; kernels of
 * listing l:ktemplate).  For every particle i < parts->n and every listed
 * neighbour j with r_ij < 2h, golden rule:
 *   Drho_i/Dt = sum_j m_j (u_ij . x_ij) F_ij
 *   a_i = -sum_j m_j (P_i/rho_i^2 + P_j/rho_j^2 + Pi_ij) x_ij F_ij
 * Landrini-Morris:
 *   Drho_i/Dt = sum_j (rho_i/rho_j) m_j (u_ij . x_ij) F_ij
 *   a_i = -sum_j m_j ((P_i + P_j)/(rho_i rho_j) + Pi_ij) x_ij F_ij
 * plus the laminar term of visc_model and the density diffusion term of
 * delta, with F of params->kernel (Wendland: F = 105/(128 pi h^5) (q - 2)^3).
 * Every combination of kernel, formulation, laminar term and diffusion is a
 * compiled instance of its own.  Gravity is excluded.
 * forces: device float[capacity][4], xyz = a_i [m/s^2], w = Drho_i/Dt,
 * fully overwritten for i < n.  Particles are read in the order of the last
 * build; positions may have drifted since (lists are reused).
 * cell_start / cell_end / neibs_brick: the cell ranges and brick-local
 * lists written by that build (device int32[n_cells] each and
 * uint16[sph_neib_brick_entries(capacity, max_neibs)]), or all NULL.  With
 * them the derivatives are computed brick by brick of cells, the particles of
 * a brick and of its one-cell halo staged in LDS with positions relative to
 * the brick's centre cell; without them one lane per particle gathers its
 * neighbours from global memory with the separation of the list predicate.
 * The two differ by rounding only (the separation of the brick form carries
 * an error of a few ulp of 2.5 cell sizes instead of one ulp of a cell size);
 * neither is bit-exact against the other.
 * In the brick form only the bricks of the build's table (those where a
 * particle has a non-empty list) are staged, the equation of state is
 * evaluated as particles are staged, and the zero derivatives of particles
 * with an empty list are written without staging: no pass over the particles
 * precedes the brick kernel.
 * workspace: device buffer of sph_forces_workspace_bytes(capacity, n_cells)
 * bytes (the per-particle equation-of-state terms of the gather form and
 * the brick counter of the persistent brick kernel, set within every call;
 * its contents on entry do not change any result).  Calls that share a workspace must not overlap.
 * Errors: SPH_ERR_ARG (also for an unknown kernel, formulation or
 * visc_model, a negative or non-finite delta, or delta > 0 without
 * parts->info), SPH_ERR_WORKSPACE. */
sph_status sph_forces(const sph_grid *grid, const sph_params *params, const sph_particles *parts,
                      const uint32_t *neibs, const uint32_t *neib_count, int32_t max_neibs,
                      const int32_t *cell_start, const int32_t *cell_end,
                      const uint16_t *neibs_brick, float *forces, void *workspace,
                      size_t workspace_bytes, void *stream);

/* Bytes of device workspace sph_forces needs (n_cells: cells of the grid). */
size_t sph_forces_workspace_bytes(int32_t capacity, int32_t n_cells);

/* Bytes of the fixed device scratch of sph_forces_noalloc (64 MiB). */
#define SPH_NOALLOC_SCRATCH_BYTES (64u << 20)

/* sph_forces for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same derivatives, from the same kernels, with the workspace taken from a
 * fixed scratch array of SPH_NOALLOC_SCRATCH_BYTES that the library holds on
 * each device it runs on (from module load to the end of the process).
 * Arguments are those of sph_forces without the workspace; the caller still
 * passes inputs and outputs.  The call allocates nothing: no hipMalloc, no
 * hipFree, no allocating library routine; the first call on a device looks
 * up the scratch array's device address (hipGetSymbolAddress) and keeps it.
 * Every call on a device shares that device's scratch, which keeps the last
 * call's contents (no result depends on them); calls that overlap on one
 * device, on different streams, race and must not be issued.
 * Errors: those of sph_forces, and SPH_ERR_SCRATCH, before any device call,
 * when sph_forces_workspace_bytes(parts->capacity, cells of the grid)
 * exceeds SPH_NOALLOC_SCRATCH_BYTES (about 8.3M particles). */
sph_status sph_forces_noalloc(const sph_grid *grid, const sph_params *params, const sph_particles *parts,
                              const uint32_t *neibs, const uint32_t *neib_count, int32_t max_neibs,
                              const int32_t *cell_start, const int32_t *cell_end,
                              const uint16_t *neibs_brick, float *forces, void *stream);

/* Explicit midpoint predictor/corrector (section "Code structure": phases
 * with dt/2 and dt).  d_dt: device double, the step.
 *   stage 0: out = state_n + dt/2 * (u_n, a_n + g, Drho_n)
 *   stage 1: out = state_n + dt   * (u*,  a*  + g, Drho*), vel_star = u*
 *            (device float[capacity][4], the stage-0 velocities); if
 *            d_time is not NULL the corrector adds dt to it (device double).
 * Offsets advance with the velocity; boundary particles only advance
 * density; dropped particles (cell < 0) are left unchanged.  `out` may
 * alias `state_n` (elementwise update).  Only out->pos and out->vel are
 * written; cell and info are read from state_n.
 * Errors: SPH_ERR_ARG. */
sph_status sph_integrate(const sph_params *params, int32_t stage, const double *d_dt,
                         const sph_particles *state_n, const float *vel_star,
                         const float *forces, sph_particles *out, double *d_time,
                         void *stream);

/* The corrector half of the step in one pass (section "Code structure": the
 * corrector's derivatives at the predicted state, then its update with dt):
 * the derivatives of `star` exactly as sph_forces computes them (same
 * lists, kernels and rounding), and, for each particle as soon as its
 * derivatives are finished, sph_integrate stage 1 applied to state_n in
 * place with vel_star = star->vel.  The result is bit for bit that of
 *   sph_forces(star) -> forces;  sph_integrate(1, state_n, star->vel, forces,
 *                                              out = state_n, d_time)
 * without the round trip of the derivatives through device memory.
 * d_dt: device double, the step; d_time: device double advanced by dt, or
 * NULL; forces: device float[capacity][4] that also receives the
 * derivatives, or NULL.  state_n->cell and ->info give each particle's
 * cell (dropped particles, cell < 0, are left unchanged) and type; only
 * state_n->pos and ->vel are written.  state_n and star hold the same
 * particles in the same order (those of the last build) and must not share
 * pos or vel storage: the kernel reads the staged state of other particles
 * while it rewrites state n.
 * Every other argument is that of sph_forces.  One step for every particle
 * (sph_forces_corrector_scenes takes one per scene).
 * Errors: those of sph_forces; SPH_ERR_ARG for a null d_dt, star or
 * state_n, state_n->n != star->n, missing state_n arrays, or shared
 * pos / vel storage. */
sph_status sph_forces_corrector(const sph_grid *grid, const sph_params *params, const sph_particles *star,
                                const uint32_t *neibs, const uint32_t *neib_count, int32_t max_neibs,
                                const int32_t *cell_start, const int32_t *cell_end,
                                const uint16_t *neibs_brick, const double *d_dt, sph_particles *state_n,
                                double *d_time, float *forces, void *workspace, size_t workspace_bytes,
                                void *stream);

/* sph_forces_corrector with a step per scene (scenes sharing one grid, see
 * sph_step_dt_scenes): a particle advances with d_dt[s] of its cell's scene
 * s (d_dt: device double[n_scenes]) and d_time[s] (device double[n_scenes],
 * or NULL) advances by d_dt[s]; a particle in a cell of no scene is left
 * as it is.  Bit for bit sph_forces followed by sph_integrate_scenes(stage
 * 1).  cell_scene, n_scenes: as for sph_integrate_scenes.  Errors: those of
 * sph_forces_corrector, and SPH_ERR_ARG for a missing scene table or
 * n_scenes outside [1, SPH_MAX_SCENES]. */
sph_status sph_forces_corrector_scenes(const sph_grid *grid, const sph_params *params,
                                       const sph_particles *star, const uint32_t *neibs,
                                       const uint32_t *neib_count, int32_t max_neibs,
                                       const int32_t *cell_start, const int32_t *cell_end,
                                       const uint16_t *neibs_brick, const double *d_dt,
                                       const int32_t *cell_scene, int32_t n_scenes, sph_particles *state_n,
                                       double *d_time, float *forces, void *workspace, size_t workspace_bytes,
                                       void *stream);

/* Reverse of sph_integrate (the transpose of its linear update; dt is held
 * fixed).  All grad arrays are device float[capacity][4] laid out like the
 * state: grad_pos xyz = dL/d(offset), grad_vel xyz = dL/du, w = dL/drho;
 * grad_forces xyz = dL/da, w = dL/d(Drho/Dt).  One reverse step is
 *   sph_integrate_backward(stage 1)   grad_pos/grad_vel = dL/dy^{n+1} on entry
 *   sph_forces_backward(y*, accumulate into grad_pos_star/grad_vel_star)
 *   sph_integrate_backward(stage 0)
 *   sph_forces_backward(y^n, accumulate into grad_pos/grad_vel)
 * after which grad_pos/grad_vel hold dL/dy^n.
 *   stage 1: writes grad_forces = (dt dL/du^{n+1} (fluid), dt dL/drho^{n+1})
 *            and initialises grad_pos_star = 0, grad_vel_star = (dt dL/do^{n+1}
 *            (fluid), 0); grad_pos/grad_vel are left as they are.
 *   stage 0: adds dL/dy* (grad_pos_star/grad_vel_star) to grad_pos/grad_vel,
 *            plus dt/2 dL/do* to the fluid velocity adjoint, and writes
 *            grad_forces = (dt/2 dL/du* (fluid), dt/2 dL/drho*).
 * Boundary particles carry no velocity update; dropped particles (cell < 0)
 * get a zero upstream.  Errors: SPH_ERR_ARG. */
sph_status sph_integrate_backward(const sph_params *params, int32_t stage, const double *d_dt,
                                  const sph_particles *state_n, float *grad_pos, float *grad_vel,
                                  float *grad_pos_star, float *grad_vel_star, float *grad_forces,
                                  void *stream);

/* Bytes of device workspace sph_forces_backward needs (n_cells: cells of
 * the grid). */
size_t sph_forces_backward_workspace_bytes(int32_t capacity, int32_t n_cells);

/* Adjoint of sph_forces with the lists held fixed.  Given grad_forces
 * (xyz = dL/da_i, w = dL/d(Drho_i/Dt)), computes dL/d(offset_i) into
 * grad_pos (xyz; w is left unchanged), dL/du_i and dL/drho_i into grad_vel,
 * and dL/d(alpha, c0, nu) into grad_params (device double[3]).  With
 * accumulate != 0 every output is added to, otherwise overwritten.
 * Atomic-free and deterministic: each particle gathers over its own list the
 * terms of the pairs where it is the central and where it is the neighbour
 * (the list is symmetric); parameter sums are reduced in double in a fixed
 * order.  The derivative of the artificial-viscosity switch at u.x = 0 is
 * that of the active branch.
 * cell_start / cell_end / neibs_brick: as for sph_forces (all three from the
 * build of the lists, or all NULL).  With them the adjoint is computed brick
 * by brick of cells from LDS (each brick in two halves along y); without them
 * one lane per particle gathers from global memory.  The two agree to
 * rounding; the brick form skips the bricks without a pair as sph_forces
 * does.  workspace: sph_forces_backward_workspace_bytes(capacity, n_cells)
 * (its contents on entry do not change any result).  Every kernel, formulation and laminar term of sph_forces is
 * differentiated, and the density diffusion term (params->delta) too; its
 * coefficient enters dL/dc0, the laminar terms dL/dnu.  Errors: SPH_ERR_ARG
 * (as for sph_forces, and for a grid with a per-cell alpha table),
 * SPH_ERR_WORKSPACE. */
sph_status sph_forces_backward(const sph_grid *grid, const sph_params *params,
                               const sph_particles *parts, const uint32_t *neibs,
                               const uint32_t *neib_count, int32_t max_neibs,
                               const int32_t *cell_start, const int32_t *cell_end,
                               const uint16_t *neibs_brick, const float *grad_forces, float *grad_pos,
                               float *grad_vel, double *grad_params, int32_t accumulate, void *workspace,
                               size_t workspace_bytes, void *stream);

/* dst[perm[k]] = src[k] for k < n, float4 records (carries an adjoint back
 * across a rebuild, see sph_build_neighbors).  src and dst must differ.
 * Errors: SPH_ERR_ARG. */
sph_status sph_unpermute(int32_t n, const uint32_t *perm, const float *src, float *dst, void *stream);

/* Bytes of device workspace sph_reduce_diagnostics needs. */
size_t sph_diagnostics_workspace_bytes(void);

/* Global conservation diagnostics in double precision (the step itself is
 * float32; only these sums and the time accumulator are double), over
 * particles i < n with cell >= 0, written to d_out (device double[12]):
 *   [0] sum m            [1..3] sum m u (fluid)   [4..6] sum m a (forces xyz,
 *   all particles; the raw pair sums are antisymmetric, so without boundary
 *   particles this is zero up to float32 rounding of the terms)
 *   [7] sum m / rho      [8] fluid count           [9] boundary count
 *   [10] max |rho/rho0 - 1| over fluid               [11] sum m |u|^2 / 2 (fluid)
 * forces may be NULL (then [4..6] = 0).  Fixed-order reduction: the result
 * is reproducible bit for bit.  Errors: SPH_ERR_ARG, SPH_ERR_WORKSPACE. */
sph_status sph_reduce_diagnostics(const sph_params *params, const sph_particles *parts,
                                  const float *forces, double *d_out, void *workspace,
                                  size_t workspace_bytes, void *stream);

/* Bytes of device workspace sph_step_dt needs. */
size_t sph_dt_workspace_bytes(void);

/* Adaptive time step kept on the device (section "The GPU in GPUSPH": the
 * step is a device reduction):
 *   dt = cfl * min(h / max c_i, sqrt(h / max |a_i + g|) [, 0.125 h^2 / nu])
 * over fluid particles i < n with cell >= 0, c_i the sound speed at rho_i,
 * evaluated in double from float32 maxima and written to d_dt (device
 * double).  forces: the derivatives of this state.
 * Errors: SPH_ERR_ARG, SPH_ERR_WORKSPACE. */
sph_status sph_step_dt(const sph_params *params, const sph_particles *parts, const float *forces,
                       double *d_dt, void *workspace, size_t workspace_bytes, void *stream);

/* Scenes that share one grid (see sph_grid) advance with time steps of their
 * own, so that each evolves as it would alone.  cell_scene: device
 * int32[n_cells], the scene of each cell (indexed by cell - cell_base);
 * n_scenes in [1, SPH_MAX_SCENES].  A particle outside the grid, or in a
 * cell whose entry is outside [0, n_scenes), belongs to no scene: it counts
 * in no scene's step and sph_integrate_scenes leaves it as it is. */
#define SPH_MAX_SCENES (1 << 20)

/* Bytes of device workspace sph_step_dt_scenes needs (0 for an invalid
 * n_scenes). */
size_t sph_dt_scenes_workspace_bytes(int32_t n_scenes);

/* sph_step_dt for each scene (section "The GPU in GPUSPH": the step is a
 * device reduction, here one per scene): d_dt[s] (device double[n_scenes])
 * = cfl * min(h / max c_i, sqrt(h / max |a_i + g|) [, 0.125 h^2 / nu]) over
 * the fluid particles i of scene s, the maxima taken in float32 as in
 * sph_step_dt (equal, bit for bit, to sph_step_dt on the scene alone); a
 * scene with no fluid particle gets cfl * 0.125 h^2 / nu, or +inf.
 * Errors: SPH_ERR_ARG, SPH_ERR_WORKSPACE. */
sph_status sph_step_dt_scenes(const sph_grid *grid, const sph_params *params, const sph_particles *parts,
                              const float *forces, const int32_t *cell_scene, int32_t n_scenes,
                              double *d_dt, void *workspace, size_t workspace_bytes, void *stream);

/* sph_integrate with a step per scene: a particle advances with d_dt[s] of
 * its scene s (d_dt: device double[n_scenes]); the corrector adds d_dt[s]
 * to d_time[s] (device double[n_scenes]) when d_time is not NULL.
 * Otherwise as sph_integrate.  Errors: SPH_ERR_ARG. */
sph_status sph_integrate_scenes(const sph_grid *grid, const sph_params *params, int32_t stage,
                                const double *d_dt, const int32_t *cell_scene, int32_t n_scenes,
                                const sph_particles *state_n, const float *vel_star,
                                const float *forces, sph_particles *out, double *d_time,
                                void *stream);

/* Number of listed pairs (i, j), i < n, whose float32 squared separation
 * (evaluated as in the neighbour predicate) is below (2h)^2 in float32:
 * the interactions sph_forces evaluates.  d_count: device uint64,
 * overwritten.  Errors: SPH_ERR_ARG. */
sph_status sph_count_interactions(const sph_grid *grid, const sph_params *params,
                                  const sph_particles *parts, const uint32_t *neibs,
                                  const uint32_t *neib_count, int32_t max_neibs,
                                  unsigned long long *d_count, void *stream);

/* Pairs missed by reused lists (section "Optimizing the neighbors search":
 * the list is built with a search radius above the kernel support so that
 * it can serve several steps; section "Too much of a good thing?": rebuilt
 * every 10 steps).  A pair that came within 2h while the lists were reused,
 * but was not listed, was left out of the derivatives.  Counted at each
 * rebuild, in two calls on the same state:
 *   phase 0, just before sph_build_neighbors, with the lists about to be
 *            replaced: d_missed[0] = their pairs with r < 2h at the current
 *            positions (as sph_count_interactions);
 *   phase 1, just after it, with the new lists: d_missed[1] = their pairs
 *            with r < 2h, which are all the pairs within 2h when no list
 *            overflowed; d_missed[2] = d_missed[1] - d_missed[0], the pairs
 *            within 2h the previous lists did not hold; d_missed[3] +=
 *            d_missed[2] (a running total the caller zeroes).
 * Both counts evaluate the separation as the neighbour predicate does, each
 * on its own encoding (the re-binning moves offsets by whole cells), so a
 * pair within rounding of 2h may be counted by one and not the other;
 * particles dropped by the rebuild lose their pairs, which can make
 * d_missed[2] negative.  d_missed: device int64[4].
 * Errors: SPH_ERR_ARG (also for a phase other than 0 or 1). */
sph_status sph_count_missed_pairs(const sph_grid *grid, const sph_params *params,
                                  const sph_particles *parts, const uint32_t *neibs,
                                  const uint32_t *neib_count, int32_t max_neibs, int32_t phase,
                                  long long *d_missed, void *stream);

/* Stream copy of `bytes` bytes from src to dst (device, 16-byte aligned,
 * bytes a multiple of 16, not overlapping), blocks_per_cu workgroups of 256
 * lanes per compute unit (1..64), each lane moving 16-byte vectors with
 * four loads in flight and nontemporal stores.  A measurement aid, no part
 * of the method: the bench times it to report the HBM bandwidth a plain
 * stream achieves on the GPU beside the data-sheet peak.
 * Errors: SPH_ERR_ARG. */
sph_status sph_stream_copy(const void *src, void *dst, size_t bytes, int32_t blocks_per_cu, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SPH_H */
