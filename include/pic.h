/*
 * pic.h - C ABI of the MI355X (gfx950) hot path of the explicit relativistic
 * particle-in-cell cycle of Melzani et al., "Apar-T" (arXiv:1308.5892).
 *
 * One step is the leap-frog cycle of App. A.3.1: field gather from the
 * staggered Yee grid (App. A.3.3), relativistic Boris push and move (App. A.3.3,
 * eq. mover), charge-conserving volume-weighting current deposit (App. A.1 and
 * A.3.4, eq. current_dep) and the Yee update of b and e (App. A.3.2), with
 * periodic boundaries (App. A.4).  The current filter of item 10 (App. A.3.4) is
 * optional (PIC_FILTER_CURRENT).
 *
 * Units are the paper's normalised ones (App. A.2): lengths in cells (dx = 1),
 * times in X0/c, e and b = cB in m_e c^2/(e X0), u = gamma v / c.  Species s has
 * charge q_s = +-e (Sect. 2.1) and mass m_s; it moves with k_s = (q_s/e)(m_e/m_s)
 * and feeds e through alpha_s = 2 sgn(q_s) / (n_x^2 rho0) (App. A.2, eq. alpha).
 *
 * State and time levels follow App. A.3.1: between calls the library holds
 * positions x and e at time t, momenta u and b at t - dt/2.
 *
 * Grid layout (App. A.3.2, A.3.3): box of n[0] x n[1] x n[2] cells, nodes at
 * integer points; e_x[i,j,k] at (i+1/2, j, k), e_y at (i, j+1/2, k), e_z at
 * (i, j, k+1/2); b_x at (i, j+1/2, k+1/2), b_y at (i+1/2, j, k+1/2), b_z at
 * (i+1/2, j+1/2, k); j_c where e_c sits.  Host field arrays are FP64,
 * component-major, cell index i + n0 (j + n1 k): value (c, i, j, k) at
 * [c * n0 n1 n2 + i + n0 (j + n1 k)].
 *
 * Memory and ownership: the caller allocates ONE device buffer (the arena, size
 * from pic_plan, 256-byte aligned) and owns the HIP stream; the library carves
 * all device state out of the arena, allocates no device memory itself, and
 * enqueues all work on that stream.  Both must outlive the context.  Host
 * buffers passed to get/set calls belong to the caller and are copied.
 *
 * Errors: every call returns PIC_OK (0) or a negative PIC_E* code;
 * pic_last_error(ctx) gives a message for the last failure on that context.
 * Kernels record faults (non-finite momentum, lost particle) in a device flag
 * word that the next pic_diag or pic_sync reports as PIC_EFLAG.
 *
 * Limits: n[0], n[1] <= 2048, n[2] <= 1024; tile edges are powers of two
 * between 1 and 8, and the tile's push workgroup must fit in LDS (8x8x8 does
 * not); at most PIC_MAX_SPECIES species; fewer than 2^29 particle
 * slots (capacity x headroom, plus 32 per tile and the overflow region) per
 * species per box; dt < 1/sqrt(3) (3-D Courant bound of the Yee scheme;
 * dt < 2/sqrt(14) with PIC_FARADAY4).
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_OK        0
#define PIC_EINVAL   (-1)  /* bad argument or configuration */
#define PIC_ECOURANT (-2)  /* dt violates a stability bound (App. B) */
#define PIC_ENOMEM   (-3)  /* arena too small or particle capacity exceeded */
#define PIC_EDEVICE  (-4)  /* a HIP runtime call failed */
#define PIC_EFLAG    (-5)  /* a kernel raised the device error flag */
#define PIC_ESTATE   (-6)  /* call not valid in the current state */

#define PIC_MAX_SPECIES 4

/* pic_config.flags */
#define PIC_FP64_FORM 1u   /* FP64 storage and arithmetic, FP64 atomics (reference form) */
#define PIC_TRACK_IDS 2u   /* carry a 32-bit particle id (parity and checkpoints) */
#define PIC_FILTER_CURRENT 4u  /* smooth the current before it enters e (App. A.3.4, last
                                  paragraph: weight 1 for the value itself, 1/2 for the 6 face,
                                  1/4 for the 12 edge and 1/8 for the 8 corner neighbours,
                                  normalised to one); the Gauss residual of pic_diag then uses
                                  the charge smoothed the same way */
#define PIC_FARADAY4 8u        /* fourth-order field solver against numerical Cerenkov emission
                                  (App. A.3.2, last paragraph; App. B, third item): Faraday's law
                                  takes the staggered fourth-order difference along each axis,
                                  (9/8)(f[+1/2] - f[-1/2]) - (1/24)(f[+3/2] - f[-3/2]); Ampere's law
                                  keeps the second-order curl, so Gauss's law holds as with Yee.
                                  Vacuum dispersion: (2/dt)^2 sin^2(w dt/2) = sum_a [4 sin^2(k_a/2)
                                  + (2/3) sin^4(k_a/2)]; Courant bound dt < 2/sqrt(14) = 0.5345;
                                  not with walls */

/* pic_load_desc.profile */
#define PIC_PROFILE_UNIFORM 0
#define PIC_PROFILE_HARRIS  1

/* device error flag bits, reported through pic_diag_out.flags */
#define PIC_FLAG_NONFINITE 1u  /* a momentum became NaN, infinite or larger than 1e15 */
#define PIC_FLAG_LOST      2u  /* a tile segment and the overflow region were full */

typedef struct pic_species {
    double q_over_e;   /* +1 or -1 (Sect. 2.1: superparticles of ions or electrons) */
    double m_over_me;  /* mass in electron masses */
} pic_species;

typedef struct pic_box {
    int32_t n[3];                             /* cells per axis */
    double  n_x;                              /* cells per reference skin depth (Sect. 2.2.1) */
    double  rho0;                             /* reference superparticles per cell, all species (eq. neandrho) */
    int64_t max_particles[PIC_MAX_SPECIES];   /* capacity per species */
    int32_t tile[3];                          /* tile edge per axis, power of two in [1, 8]; 0 = 4 */
    int32_t walls;                            /* 0: periodic; 1 + a: perfectly conducting walls at the
                                                 two faces normal to axis a (App. A.4: normal b and
                                                 tangential e vanish on the wall plane, particles are
                                                 reflected; both faces share the node plane of index 0
                                                 along a); n[a] >= 2; not with PIC_FILTER_CURRENT */
} pic_box;

typedef struct pic_config {
    int32_t            n_boxes;     /* independent periodic boxes advanced together */
    const pic_box     *boxes;       /* n_boxes entries (copied) */
    int32_t            n_species;   /* same species list in every box */
    pic_species        species[PIC_MAX_SPECIES];
    double             dt;          /* time step in X0/c */
    int32_t            sort_interval;  /* steps between counting-sort repacks; 0 = never */
    uint32_t           flags;       /* PIC_FP64_FORM | PIC_TRACK_IDS | PIC_FILTER_CURRENT | PIC_FARADAY4 */
    int32_t            hist_bins;   /* bins of the log10(gamma-1) histogram in pic_diag (0 = none) */
    double             hist_lo, hist_hi;   /* histogram range of log10(gamma - 1) */
    double             headroom;    /* particle slots per particle (>= 1.05; 0 = 1.3) */
} pic_config;

/* One drifting Maxwell-Juttner population (Sect. 4.3, eq. Jutt). */
typedef struct pic_mj {
    double  theta;        /* T / (m_s c^2) */
    double  gamma_beta;   /* signed Gamma0 beta0 of the drift (0: at rest) */
    int32_t axis;         /* drift axis 0, 1, 2 */
} pic_mj;

/*
 * A load of co-located pairs (Sect. 2.1): species_a and species_b particles on
 * top of each other so that the charge density stays zero, momenta drawn from
 * two drifting Maxwell-Juttner distributions (Sect. 4.3; App. D).  ppc is the
 * number of pairs per cell at the profile's peak in the simulation frame.
 * UNIFORM: round(ppc * cells) pairs, positions uniform in the box.  HARRIS:
 * density ~ 1/cosh^2((s - centre)/thickness) along profile_axis (App. C) on the
 * window |s - centre| < half_width, round(ppc * (cells/n[axis]) * 2 thickness
 * tanh(half_width/thickness)) pairs, other coordinates uniform.
 * Random numbers: Philox4x64-10 with key (seed, stream) and counter
 * (pair, j, 0, 0); the mapping of the twelve words per pair is fixed.
 */
typedef struct pic_load_desc {
    int32_t  box;
    int32_t  species_a, species_b;
    pic_mj   mj_a, mj_b;
    double   ppc;
    int32_t  profile;         /* PIC_PROFILE_UNIFORM or PIC_PROFILE_HARRIS */
    int32_t  profile_axis;
    double   centre, thickness, half_width;
    uint64_t seed, stream;
} pic_load_desc;

/* Harris-sheet magnetic field (App. C, eq. B_field_Harris) on one box. */
typedef struct pic_harris_field {
    int32_t box;
    int32_t grad_axis;   /* axis along which the field varies */
    int32_t field_axis;  /* component of b that is set (!= grad_axis) */
    int32_t n_sheets;    /* 1: b = b0 tanh((s-c0)/L); 2: b = b0 [tanh((s-c0)/L) - tanh((s-c1)/L) - 1] */
    double  b0, thickness;
    double  centre[2];
} pic_harris_field;

typedef struct pic_diag_out {
    double  t;                          /* simulation time of x and e */
    int64_t step;
    double  W_E[3], W_B[3];             /* (1/alpha0) sum_cells e_c^2/2 and (b^t)_c^2/2 */
    double  K[PIC_MAX_SPECIES];         /* sum (m_s/m_e)(gamma^t - 1) */
    double  P[PIC_MAX_SPECIES][3];      /* sum of u^- = u^{t-dt/2} + (k dt/2) E(x^t) */
    double  sum_gm1[PIC_MAX_SPECIES];   /* sum (gamma^t - 1) */
    int64_t n_particles[PIC_MAX_SPECIES];
    int64_t n_overflow[PIC_MAX_SPECIES];   /* particles in the overflow region */
    double  gauss_max, gauss_rms;       /* |div e - rho| over the nodes, rho = sum alpha_s W(x_p) */
    uint32_t flags;                     /* PIC_FLAG_* raised since the last report */
} pic_diag_out;

typedef struct pic_ctx pic_ctx;

/*
 * Size of the device arena that pic_init needs for cfg.  Validates cfg;
 * returns PIC_EINVAL with *arena_bytes untouched on a bad configuration.
 */
int pic_plan(const pic_config *cfg, size_t *arena_bytes);

/*
 * Create a context.  dev_arena: device pointer of at least pic_plan bytes
 * (borrowed).  hip_stream: hipStream_t to enqueue on (borrowed; NULL = default).
 * Checks the 3-D Courant bound dt < 1/sqrt(3) (App. B states the bound as
 * dt < X0/sqrt 2, which is the 2-D one) and omega_pe dt = dt/n_x < 2 (App. B),
 * returning PIC_ECOURANT.  Zeroes all fields and particles.
 */
int pic_init(const pic_config *cfg, void *dev_arena, size_t bytes, void *hip_stream,
             pic_ctx **out);

/*
 * Load a pair population (see pic_load_desc).  FP64 on the device: inverse-CDF
 * table of the p_y marginal (App. D, eq. distr_y), Newton solve for u
 * (App. D, eq. finding_u), rounding to the storage format.  The particles are
 * binned, and their momenta integrated back by dt/2 in the fields of that
 * moment (App. A.3.1), at the next pic_step or pic_diag.  Asynchronous.
 * PIC_ENOMEM if the species capacity would be exceeded.
 */
int pic_load_maxwell_juttner(pic_ctx *ctx, const pic_load_desc *d);

/*
 * Set the Harris-sheet b (App. C) at t = 0 and shift it to the stored time
 * level: b^{-dt/2} = b^0 + (dt/2) curl e^0.  Other components are unchanged.
 */
int pic_set_harris_field(pic_ctx *ctx, const pic_harris_field *h);

/*
 * Enqueue n full cycles of App. A.3.1 on the stream for every box.  Kernel
 * faults surface in the next pic_diag / pic_sync.  Particles are re-binned
 * every sort_interval steps, and also as soon as an overflow region (the
 * slow path for particles whose tile segment is full) is half full, or holds
 * more than 8192 particles:
 * after each push the e update writes the fill of the fullest one into
 * coherent pinned host memory (a few bytes, allocated by pic_init), and
 * pic_step reads that report two steps later, so it keeps the stream at most
 * two steps ahead of the host instead of returning at once.  Which particles take the slow path depends
 * on the order of the slot claims, but it computes the same arithmetic as the
 * tile path, and the FP32 form sums the current in int64 fixed point: a run
 * of the FP32 form is bitwise reproducible.
 */
int pic_step(pic_ctx *ctx, int n);

/*
 * FP64 diagnostics of box `box` at the current time (synchronises):
 * field energies per component, kinetic energy and k = 0 momentum per species,
 * the gamma-1 histogram (hist: caller array of n_species * hist_bins int64, or
 * NULL), and the Gauss-law residual.  Returns PIC_EFLAG (after filling *out)
 * if the device error flag was raised; the flag is then cleared.
 */
int pic_diag(pic_ctx *ctx, int box, pic_diag_out *out, int64_t *hist);

/*
 * For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): pic_diag with the
 * same arguments and results, whose accumulators, charge density and
 * histogram live in a static device array of the library (32 MiB per GPU,
 * held until the process ends; its device address is taken by pic_init)
 * instead of the context's arena.  It calls no allocator, and clears what
 * it sums with kernels (no memset).  The box may need at most 32 MiB:
 * 8 bytes per cell plus about 2 KiB, so about 4.1 M cells; a larger box gives
 * PIC_ENOMEM.  Particles loaded or set since the last pic_step / pic_diag are
 * not binned by this call: it returns PIC_ESTATE then.  Every context on one
 * GPU shares the array, so calls that overlap on one GPU (different
 * streams or threads) race; calls on one stream are ordered.  Synchronises.
 */
int pic_diag_noalloc(pic_ctx *ctx, int box, pic_diag_out *out, int64_t *hist);

/*
 * Copy particles of (box, species) to the host as FP64: x[3n] absolute
 * positions in [0, n_axis), u[3n], id[n] (NULL allowed; zeros without
 * PIC_TRACK_IDS).  *n: in = capacity of the arrays, out = particle count
 * (PIC_ENOMEM if too small).  With PIC_TRACK_IDS the output is ordered by id.
 * Synchronises.
 */
int pic_get_particles(pic_ctx *ctx, int box, int species, double *x, double *u,
                      int32_t *id, int64_t *n);

/*
 * Replace all particles of (box, species) by n given ones (x^t, u^{t-dt/2};
 * no half step is applied).  Positions are wrapped into the box and rounded to
 * the storage format.  id may be NULL (ids 0..n-1).
 */
int pic_set_particles(pic_ctx *ctx, int box, int species, const double *x, const double *u,
                      const int32_t *id, int64_t n);

/* Copy e^t, b^{t-dt/2} and the pending current (NULLs allowed) to the host. */
int pic_get_fields(pic_ctx *ctx, int box, double *e, double *b, double *j);

/*
 * Set e^t and b^{t-dt/2} of a box (NULL leaves that field unchanged).  In a
 * box with walls the tangential e and the normal b on the wall plane are set
 * to zero, the conductor's condition (App. A.4).
 */
int pic_set_fields(pic_ctx *ctx, int box, const double *e, const double *b);

/* Kernel timing of pic_step, from HIP events recorded on the context's stream
 * right before and after each launch (measurement hook, off by default). */
typedef struct pic_timing {
    int64_t push_launches;   /* fused gather + push + deposit kernel */
    double  push_ms;
    int64_t field_launches;  /* Yee b and e updates (one pair per step) */
    double  field_ms;
    int64_t sort_launches;   /* counting-sort repacks */
    double  sort_ms;
} pic_timing;

/* Event recording in pic_step: 0 off, 1 around every push, field update and
 * repack, 2 around the push only (fewer events in the stream; each costs a
 * few microseconds of the step).  Other values: PIC_EINVAL. */
int pic_set_timing(pic_ctx *ctx, int enable);

/* Sum the recorded intervals into *out (synchronises); reset != 0 forgets them. */
int pic_get_timing(pic_ctx *ctx, pic_timing *out, int reset);

/* Wait for the stream; returns PIC_EFLAG if the device error flag is set. */
int pic_sync(pic_ctx *ctx);

/* Number of completed steps. */
int64_t pic_steps_done(const pic_ctx *ctx);

/* Release the context (the arena and stream stay the caller's). */
int pic_free(pic_ctx *ctx);

/* Message of the last error on ctx (static storage of the context). */
const char *pic_last_error(const pic_ctx *ctx);

/*
 * Fourier power spectrum of one field component in the planes normal to
 * `normal_axis`, summed over those planes (Sect. 3.2.2, method of
 * measurement): PS(m1, m2) = sum_p |sum_{i1,i2} f(i1, i2, p)
 * exp(-2 pi i (m1 i1 / N1 + m2 i2 / N2))|^2, where (a1, a2) are the two other
 * axes in increasing order, N1 = n[a1], N2 = n[a2], and f is e^t (field 0) or
 * b^t = b^{t-dt/2} - (dt/2) curl e^t (field 1), component comp, at its Yee
 * position.  FP64.  ps: caller's host array of N1 * N2 doubles, mode (m1, m2)
 * at ps[m1 + N1 m2] for m1 in [0, N1), m2 in [0, N2) (the paper samples
 * m1 <= N1/2, m2 <= N2/2).  Synchronises.
 */
int pic_field_spectrum(pic_ctx *ctx, int box, int field, int comp, int normal_axis, double *ps);

/* Outcome of pic_autotune. */
typedef struct pic_tune_result {
    double  ms_per_step;          /* time per step of the chosen configuration */
    double  ms_per_step_default;  /* time per step of cfg as given */
    int32_t trials;               /* configurations timed */
} pic_tune_result;

/*
 * Tile shape and sort interval by measurement (not part of the paper's
 * method; the work split of this library).  Boxes are grouped by particle
 * capacity per cell (below 32, below 128, above); for each group in turn the
 * tile shapes 4x4x4, 8x4x4 and 8x8x4 are tried on the whole configuration,
 * keeping the fastest, then the sort interval among 25, 50, 100, 200 and
 * cfg's.
 * Each trial creates a context in dev_arena (borrowed, 256-byte aligned,
 * `bytes` long; size it with pic_plan for cfg with its smallest tiles),
 * applies the n_loads loads, runs steps/2 warm-up and `steps` timed steps on
 * hip_stream, and frees the context; trials that do not fit the arena are
 * skipped.  On PIC_OK, boxes_out (cfg->n_boxes entries, caller-owned) holds the
 * boxes with the chosen tiles and *cfg_out the configuration, its boxes
 * pointer set to boxes_out.  Synchronises; leaves no state behind.
 */
int pic_autotune(const pic_config *cfg, const pic_load_desc *loads, int n_loads, void *dev_arena, size_t bytes,
                 void *hip_stream, int steps, pic_config *cfg_out, pic_box *boxes_out, pic_tune_result *res);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H */
