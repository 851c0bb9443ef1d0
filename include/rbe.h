/*
 * rbe.h -- C ABI of the random batch Ewald (RBE) Fourier-space step on one
 * AMD Instinct MI355X (gfx950).
 *
 * The method (Liang, Tan, Hong, Jin, Xu, Li, "A random batch Ewald method for
 * charged particles in the isothermal-isobaric ensemble", arXiv:2110.14362):
 *   - section 4.1, eq. (U1fourier): the Ewald Fourier sum over k = 2 pi h^-T m;
 *   - section 4.2, eq. (S), (psf), (probexpression): the normaliser S and the
 *     sampling law exp(-|k|^2/(4 alpha))/S over nonzero k;
 *   - section 4.2, eq. (appforce) and (apppress): the batch estimators of the
 *     Fourier-space force and pressure with weight S/p;
 *   - appendix C, eq. (pressuretensorflexible) and (pressurerect): the
 *     pressure tensor, and the per-axis sampling of a rectangular cell.
 *
 * Conventions shared by every entry point
 *   - Units: the caller's.  `coulomb` is the Coulomb constant C (1 in reduced
 *     units, 332.0637 kcal A/(mol e^2) in "real" units).  `alpha` is the
 *     paper's splitting parameter: the kernel splits as erf(sqrt(alpha) r)/r,
 *     so alpha has units of 1/length^2 (for g = 0.3/A, alpha = 0.09/A^2).
 *   - Cell: orthorhombic, h = diag(lx, ly, lz), V = lx*ly*lz.  Positions may
 *     lie outside [0, l); they are used modulo the cell.
 *   - Particle arrays are structure-of-arrays FP64 DEVICE pointers owned by the
 *     caller (x, y, z, fx, fy, fz: n doubles each, no alignment beyond 8 B).
 *   - The context owns all its device scratch, allocated once in rbe_init.
 *     No other entry point allocates device memory.
 *   - Work is queued on the context's HIP stream and returns without waiting,
 *     except where an argument is a HOST output pointer (the call then waits
 *     for the stream).
 *   - Errors: every entry point returns rbe_status; RBE_OK is 0.  The text of
 *     the last error of the calling thread is returned by rbe_last_error().
 *     A failed call leaves the context usable unless it says otherwise.
 *   - Thread safety: a context must not be used by two threads at once.
 */
#ifndef RBE_H
#define RBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rbe_ctx_s* rbe_ctx;

typedef enum {
  RBE_OK = 0,
  RBE_ERR_ARG = 1,         /* invalid argument (size, value, null pointer)      */
  RBE_ERR_ALLOC = 2,       /* device or host allocation failed                  */
  RBE_ERR_DEVICE = 3,      /* a HIP call failed                                 */
  RBE_ERR_STATE = 4,       /* call out of order (e.g. forces before a sample)   */
  RBE_ERR_NONNEUTRAL = 5,  /* |sum q| > 1e-10 * sum |q| (section 4.1 assumes a
                              neutral system; the k = 0 term is dropped)        */
  RBE_ERR_CAPACITY = 6     /* box grew beyond the sampler-table capacity        */
} rbe_status;

typedef enum {
  RBE_BOX_ISO = 0,      /* cubic cell, isotropic coupling (section 3.2)        */
  RBE_BOX_SEMIISO = 1,  /* lx == ly, xy and z coupled separately (appendix A)  */
  RBE_BOX_ANISO = 2,    /* any rectangular cell                                */
  /* Triclinic cell (appendix C), Fourier part only: h = [[lx, xy, xz],
     [0, ly, yz], [0, 0, lz]] (columns = cell vectors), given as 6 doubles
     (lx, ly, lz, xy, xz, yz) wherever a cell is passed from the host, with
     |xy| <= lx, |xz| <= lx, |yz| <= ly; k = 2 pi h^-T m, the sampling law
     exp(-|k|^2/(4 alpha))/S no longer factorises over the three components of
     m and is drawn exactly by rejection (rbe_sample_k).  Not with
     rbe_rescale_box_dev, the Metropolis-Hastings sampler or sample reuse
     (RBE_ERR_ARG), nor in the served batch.                                   */
  RBE_BOX_TRICLINIC = 3
} rbe_box_mode;

typedef enum {
  /* FP64 everywhere: phases, sin/cos, sums, forces, virial.                   */
  RBE_PREC_FP64 = 0,
  /* Exact phase reduction (integer part removed without rounding), FP32
     sin/cos, FP32 sums with compensation (blocked Kahan) per lane, FP64 sums
     across lanes and blocks, FP64 virial and energy, FP32 force accumulation
     over the batch with an FP64 store.                                        */
  RBE_PREC_FP32 = 1
} rbe_precision;

typedef enum {
  /* Exact independent draws of the law of eq. (probexpression) every step
     (inverse CDF per axis; the default).                                      */
  RBE_SAMPLER_EXACT = 0,
  /* Section 4.3, online approach: P Metropolis-Hastings chains, one per batch
     slot, carried from step to step; rounded continuous Gaussian proposal
     (see rbe_set_sampler).                                                    */
  RBE_SAMPLER_MH = 1
} rbe_sampler;

typedef struct {
  int64_t  n;          /* number of charges, >= 1                              */
  int32_t  p;          /* force batch size, 1..65536                          */
  int32_t  box_mode;   /* rbe_box_mode                                         */
  int32_t  precision;  /* rbe_precision                                        */
  int32_t  p_pressure; /* pressure batch size p~ (the remark after eq.
                          (apppress): it may differ from p): 0 means p~ = p,
                          else p <= p~ <= 65536.  Each step draws ONE batch of
                          p~ frequencies and forms rho for all of them; the
                          forces use its first p (weight S/p), the virial
                          tensor and the energy all p~ (weight S/p~).  Below,
                          "the batch" means these p~ frequencies.             */
  double   alpha;      /* splitting parameter (1/length^2), > 0               */
  double   coulomb;    /* Coulomb constant C, > 0                              */
  uint64_t seed;       /* Philox key word 0                                    */
  uint64_t system_id;  /* Philox key word 1                                    */
} rbe_config;

/* Create a context.
 *   cfg      : configuration (copied).
 *   d_q      : DEVICE pointer to n FP64 charges; copied into the context, so
 *              the caller may free it afterwards.  Must be neutral
 *              (RBE_ERR_NONNEUTRAL otherwise).
 *   box_host : HOST pointer to (lx, ly, lz) > 0 (triclinic mode: (lx, ly,
 *              lz, xy, xz, yz), see RBE_BOX_TRICLINIC).  Semi-isotropic mode
 *              needs |lx - ly| <= 1e-12 * lx.  The sampler tables are sized
 *              for side lengths up to 2x these values.
 *   stream   : hipStream_t to queue work on (NULL = default stream).
 *   out      : receives the context.
 * Waits for the stream (the neutrality check reads a device sum).  Calls
 * rbe_rescale_box(box_host) before returning. */
rbe_status rbe_init(const rbe_config* cfg, const double* d_q, const double* box_host,
                    void* stream, rbe_ctx* out);

/* Set the stream used by later calls (NULL = default stream). */
rbe_status rbe_set_stream(rbe_ctx ctx, void* stream);

/* New cell (section 4.2 eq. (S), (psf); appendix C, rectangular sampling;
 * triclinic mode: 6 values, see RBE_BOX_TRICLINIC and rbe_sample_k; S then
 * from its Poisson-summed lattice form).
 * Sets the cell from which V, the per-axis discrete-Gaussian tables
 *   w_j(m) = exp(-pi^2 m^2 / (alpha l_j^2)),  |m| <= ceil(sqrt(53 ln2 alpha) l_j / pi),
 * their running sums, H_j and S = H_x H_y H_z - 1 are computed.  box_host is
 * read immediately (host pointer, 3 doubles); the device work runs inside the
 * next kernel that needs it (normally the next rbe_forces_pressure), so a
 * rescale, a draw and an evaluation cost two kernel launches in all.
 * RBE_ERR_CAPACITY if a side exceeds 2x its value at rbe_init. */
rbe_status rbe_rescale_box(rbe_ctx ctx, const double* box_host);

/* Same as rbe_rescale_box with the cell read from DEVICE memory (3 doubles)
 * when the work runs (the next kernel that needs the cell, on the stream), so
 * a device-side barostat can feed it.  A cell outside the table capacity is
 * clamped, recorded on the device and reported by rbe_check. */
rbe_status rbe_rescale_box_dev(rbe_ctx ctx, const double* d_box);

/* Draw the batch of step `step` (section 4.2 eq. (probexpression); section
 * 4.3): the batch (p~ independent nonzero integer vectors m, p~ = p unless
 * cfg.p_pressure is set) with probability
 * exp(-|k|^2/(4 alpha))/S, k = 2 pi (mx/lx, my/ly, mz/lz), from the
 * counter-based Philox4x64-10 stream keyed by (seed, system_id) with counter
 * (step, l, 'ksam', 0) for sample l.  Triclinic cell: k = 2 pi h^-T m and
 * Q(m) = |k|^2/(4 alpha) = m^T A m; attempt a of sample l proposes m from
 * the separable law exp(-sum_j d_j m_j^2) (d = t diag(A), t = (1 - 1e-9) x
 * the smallest eigenvalue of diag(A)^-1/2 A diag(A)^-1/2, so that
 * Q(m) >= sum d_j m_j^2) with counter (step, l, 'ksam', a) and accepts it
 * with probability exp(-(Q(m) - sum d_j m_j^2)), the uniform from counter
 * (step, l, 'kacc', a); after 256 rejections the last proposal is kept.  The same step always gives the same
 * batch for the same cell.  Uses the cell of the last rescale.  Recorded here
 * and drawn inside the next rbe_forces_pressure (or by rbe_get_k). */
rbe_status rbe_sample_k(rbe_ctx ctx, uint64_t step);

/* Choose how rbe_sample_k draws the batch.  RBE_SAMPLER_MH (section 4.3,
 * online approach): chain l of the P chains keeps its frequency m_l from the
 * previous sampled step and takes `iters` (1..64) Metropolis-Hastings moves
 * towards the law of the current cell: per axis exp(-m^2/(2 sigma_j^2)),
 * sigma_j = sqrt(alpha) l_j/(pi sqrt 2), m != 0.  Proposal: z ~ N(0, sigma_j^2)
 * per axis, m'_j = floor(z + 1/2), pmf q_j(m) = Phi((m + 1/2)/sigma_j) -
 * Phi((m - 1/2)/sigma_j) (independent of the state); acceptance
 * min(1, pi(m') q(m)/(pi(m) q(m'))), m' = 0 rejected.  Randoms: Philox
 * counter (step, l, 'mhch', 2 it) -> three Box-Muller normals, (step, l,
 * 'mhch', 2 it + 1) -> the acceptance uniform.  The chains start from an
 * exact draw at the next sampled step (also after every call of this
 * function).  Drawing ahead is off under this sampler.  Allocates the chain
 * state (2 x 3p int32) on first use; waits. */
rbe_status rbe_set_sampler(rbe_ctx ctx, int32_t sampler, int32_t iters);

/* Sample reuse, the parallel strategy of section 4.3: the steps are grouped
 * in blocks [kM, (k+1)M) of the step counter, M = `period`; every draw of a
 * block uses the sampler law of the cell current at the block's first sampled
 * step (frozen then), while the forces, k vectors and S use the current cell.
 * Draw of step s: as rbe_sample_k, counter (s, l, 'ksam', 0), with the frozen
 * cell's tables, so the M batches of a block are independent and any one of
 * them can be drawn first.  period = 1 (the default) draws every step from
 * the current cell.  Exact sampler only (RBE_ERR_ARG under the MH sampler).
 * Draws then run in the standalone kernels before the step.  Allocates the
 * frozen cell's tables on first use; waits. */
rbe_status rbe_set_sample_reuse(rbe_ctx ctx, int32_t period);

/* Test hook: replace the batch by p_in host vectors h_m (p_in x 3 int32,
 * row-major, every row nonzero, |m_j| <= 2048).  p_in must equal the batch
 * size max(cfg.p, cfg.p_pressure).
 * Copies synchronously. */
rbe_status rbe_set_k(rbe_ctx ctx, const int32_t* h_m, int32_t p_in);

/* Copy the current batch (p~ x 3 int32) to host memory.  Waits. */
rbe_status rbe_get_k(rbe_ctx ctx, int32_t* h_m);

/* Fourier-space forces, virial tensor and energy of the current batch
 * (section 4.2 eq. (appforce), (apppress); appendix C eq.
 * (pressuretensorflexible) with exp(-k^2/4alpha) replaced by S/p):
 *   rho_l = sum_j q_j exp(i k_l.r_j)                       (l < p~)
 *   F_i  -= q_i sum_{l < p} c_l (cos(k_l.r_i) Im rho_l - sin(k_l.r_i) Re rho_l) k_l,
 *           c_l = C (S/p) 4 pi / (V |k_l|^2)
 *   W_ab  = C (2 pi / V)(S/p~) sum_{l < p~} |rho_l|^2/|k_l|^2
 *           [delta_ab - 2 (1/|k_l|^2 + 1/(4 alpha)) k_la k_lb]
 *   U1*   = C (2 pi / V)(S/p~) sum_{l < p~} |rho_l|^2/|k_l|^2 - C sum_i q_i^2 sqrt(alpha/pi)
 * (p~ = p unless cfg.p_pressure is set).
 * The Fourier-space pressure tensor is W / V; the scalar pressure P2* of eq.
 * (apppress) is (Wxx + Wyy + Wzz)/(3V).
 *   d_x, d_y, d_z   : DEVICE positions (n doubles each).
 *   d_fx, d_fy, d_fz: DEVICE forces (n doubles each); overwritten, or added
 *                     to when accumulate != 0.  May not alias the positions.
 *   d_virial6       : DEVICE, 6 doubles (xx, yy, zz, xy, xz, yz) written, or
 *                     NULL.
 *   d_energy        : DEVICE, 1 double (U1*) written, or NULL.
 * RBE_ERR_STATE if no batch was drawn or set since rbe_init.  Asynchronous. */
rbe_status rbe_forces_pressure(rbe_ctx ctx, const double* d_x, const double* d_y,
                               const double* d_z, double* d_fx, double* d_fy,
                               double* d_fz, int accumulate, double* d_virial6,
                               double* d_energy);

/* Copy rho of the last rbe_forces_pressure (p~ complex numbers as 2p~ doubles:
 * re0, im0, re1, ...) to host memory.  Waits. */
rbe_status rbe_get_rho(rbe_ctx ctx, double* h_rho);

/* Copy the cell-derived values of the last rescale to host memory.  Waits.
 * h_info[0..9] = V, S, Hx, Hy, Hz, lx, ly, lz, mcut_x, mcut_y (as doubles);
 * h_info[10] = mcut_z; h_info[11] = device error flags (0 = none). */
rbe_status rbe_get_box_info(rbe_ctx ctx, double* h_info);

/* Launch geometry chosen at rbe_init (no device work): h_plan[16] = X
 * (particle chunks), Y (frequency slices), KB (frequency groups per block),
 * R (frequencies per lane), GX (chunks per reduction group), NG (groups),
 * chunk (particles per chunk), Ppad, KS (force waves per particle group),
 * PW (particle waves per force block), k2reduce (1: the force kernel sums
 * the rho partials) of the two-launch form; fused (1: rbe_forces_pressure
 * runs as one launch, see rbe_set_fused); the single launch's chunks, chunk
 * size and force slices; 0. */
rbe_status rbe_get_plan(rbe_ctx ctx, int32_t* h_plan);

/* Test and measurement hook: the launch form of rbe_forces_pressure.  With
 * enable = 1 a context whose plan allows it (every particle
 * chunk within one 512-particle LDS tile, p <= 512 frequencies in one
 * block, every block resident at once: n up to about 131,000 charges on
 * MI355X) runs the whole step of section 4.2 as ONE launch: each
 * block forms its chunk's rho partial, the partials are reduced in a fixed
 * order by the last-arriving blocks, the last of which stores the force
 * constants while the other blocks wait for them on a device counter, and
 * each block then forms its own particles' forces (eq. (appforce)) from
 * positions still in LDS.  The wait is bounded (about 0.2 s); a block that
 * gives up (only possible when another application keeps some of the grid's
 * blocks off the device) skips its forces and rbe_check reports it.
 * enable = 0 (the default, measured faster on MI355X: the single launch's
 * partial sums written in the same launch must be read through the
 * coherence point, the second launch reads them through L2): two launches
 * (structure factors, then forces).
 * Both forms do the same arithmetic in the same order: identical results.
 * RBE_ERR_ARG unless enable is 0 or 1.  No device work. */
rbe_status rbe_set_fused(rbe_ctx ctx, int32_t enable);

/* Proposition 1 measured on the device (section 4.4, eq. (ForceExp),
 * (PressExp)): `batches` (2..10^6) evaluations of rbe_forces_pressure at the
 * DEVICE positions d_x, d_y, d_z and the current cell, with the batches of
 * steps first_step, first_step + 1, ... under the context's sampler; the
 * device keeps per particle and component the sums of F* and F*^2, and the
 * sums of the isotropic P2* = tr W/(3V) and of its square.  HOST outputs:
 * h_out[4] = { sum over particles of the sample variance of F*_i across
 * batches (summed over components: the total of E|chi_i|^2, eq.
 * (ForceExp)), sample variance of P2* (eq. (PressExp)), sum over particles
 * of |mean F*_i|^2, mean P2* }; h_var [n] (nullable) = the per-particle
 * sample variances.  Allocates and frees 9n + 8 doubles of device scratch:
 * a measurement call, not for time steps.  Waits.  Leaves the context's
 * batch and last results as the final evaluation left them. */
rbe_status rbe_variance_probe(rbe_ctx ctx, const double* d_x, const double* d_y,
                              const double* d_z, int32_t batches, uint64_t first_step,
                              double* h_out, double* h_var);

/* The batch size for a target variance by the 1/p law of Proposition 1
 * (eq. (ForceExp), (PressExp): the variance of a batch mean of p i.i.d.
 * draws is the one-draw variance over p): given the variance `var` measured
 * at batch size p (e.g. h_out[0] or h_out[1] of rbe_variance_probe),
 * *p_out = ceil(p var / target), clamped to 1..65536.  RBE_ERR_ARG for p < 1,
 * var < 0 or target <= 0 (or non-finite).  Host arithmetic only. */
rbe_status rbe_batch_size_for_variance(int32_t p, double var, double target, int32_t* p_out);

/* Issue rates of the current device behind the roofline peaks: FP32 sines
 * (v_sin_f32, the transcendental unit), FP32 FMAs, FP64 FMAs, and sines with
 * four FP32 FMAs beside each (whether both kinds issue side by side), from
 * eight independent chains per thread on 16 blocks of 4 waves per compute
 * unit, timed with HIP events.  h_out[5] (HOST) = {sines/s, FP32 FMAs/s,
 * FP64 FMAs/s, sines/s of the mixed kernel, compute units}.  Allocates and
 * frees two small device buffers; runs on the null stream; waits. */
rbe_status rbe_measure_issue_rates(double* h_out);

/* Wait for the stream and report device-side errors (capacity overflow of a
 * device rescale: RBE_ERR_CAPACITY; a single-launch step whose bounded wait
 * for the other blocks' partial sums gave up: RBE_ERR_DEVICE, its forces not
 * written) as a status.  Clears the device error flags. */
rbe_status rbe_check(rbe_ctx ctx);

/* Kernel timing for measurement.  While enabled, each kernel this context
 * launches carries two HIP events that the launch itself timestamps at the
 * kernel's start and end (hipExtLaunchKernel, on the context's stream: the
 * stream the kernel runs on), so queueing between launches is not counted.
 * max_launches (>= 1) bounds the launches
 * recorded per kernel kind; later launches run untimed.  0 disables and
 * releases the events.  Creates host-side HIP events only (no device memory). */
rbe_status rbe_timing_enable(rbe_ctx ctx, int32_t max_launches);

/* Wait for the stream and read the timing since the last read or enable:
 * h_ms[k] = total device milliseconds and h_count[k] = launches of kernel kind
 * k, for k = 0 standalone tables, 1 standalone draw, 2 structure factors
 * (with the reduction, virial and energy), 3 forces, 4 single-launch step
 * (rbe_set_fused); h_ms and h_count hold 5 entries.  Resets the totals
 * (timing stays enabled). */
rbe_status rbe_timing_read(rbe_ctx ctx, double* h_ms, int32_t* h_count);

/* Release the context and its device memory (waits for the stream). */
void rbe_destroy(rbe_ctx ctx);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one whole
 * Fourier-space step with no context and no allocation.  Same results, bit
 * for bit, as rbe_init(cfg, d_q, box_host) + rbe_rescale_box(box_host) +
 * rbe_sample_k(step) + rbe_forces_pressure(...) on the single-launch plan
 * (rbe_set_fused): the batch of `step` for the cell box_host (exact sampler),
 * rho, forces, virial tensor and energy.  DEVICE arrays: d_q [n] charges,
 * d_x, d_y, d_z [n], d_fx, d_fy, d_fz [n] (overwritten, or added to when
 * accumulate != 0), d_virial6 [6] and d_energy [1] (each nullable), d_rho
 * [2p~] (nullable: rho of the batch); box_host is a HOST array of 3 sides
 * (6 values for RBE_BOX_TRICLINIC).
 * stream: hipStream_t (NULL: the null stream).  Asynchronous: two kernel
 * launches, no copies, no allocation, no wait.
 * Every intermediate (the batch, partial sums, rho, force constants,
 * counters) lives in one file-scope device array of 4 MiB that each GPU the
 * library runs on keeps until the process ends; a call clears what must
 * start at zero.  Calls that overlap on one GPU (other streams, other host
 * threads) share that array and race: serialise them.
 * Limits: the single-launch plan (each particle chunk within one
 * 512-particle tile, p~ <= 512, every block resident at once: up to about
 * 131,000 charges on MI355X) and the 4 MiB; otherwise RBE_ERR_CAPACITY with
 * nothing launched.  Configuration and cell errors as rbe_init
 * (RBE_ERR_ARG); neutrality is NOT checked (it needs a device read; the
 * caller guarantees it), and device-side flags (a cell beyond the sampler
 * tables, a wait that gave up) are not reported. */
rbe_status rbe_forces_pressure_noalloc(const rbe_config* cfg, const double* d_q,
                                       const double* box_host, uint64_t step,
                                       const double* d_x, const double* d_y, const double* d_z,
                                       double* d_fx, double* d_fy, double* d_fz, int accumulate,
                                       double* d_virial6, double* d_energy, double* d_rho,
                                       void* stream);

/* ---------------------------------------------------------------------------
 * Real-space part of the Ewald split (section 4.1 eq. (U2), eq. (force) second
 * term; section 4.2: computed with the nearest image only, for pairs closer
 * than a cutoff), FP64.  For x = r_j - r_i (nearest image) and |x| < rc:
 *   U2  = (C/2) sum_{i != j} q_i q_j erfc(sqrt(alpha)|x|)/|x|
 *   F_i = -C q_i sum_j q_j G(|x|) x/|x|,
 *         G(r) = erfc(sqrt(alpha) r)/r^2 + 2 sqrt(alpha/pi) exp(-alpha r^2)/r
 *   W   = +(C/2) sum_{i != j} q_i q_j G(|x|) x x^T/|x|   (energy units)
 * The paper prints the virial term with the opposite sign; the sign here is
 * the derivative of U2 in the cell at fixed reduced coordinates.
 * Optionally a truncated Lennard-Jones term per type pair (not part of the
 * paper's method; the water- and membrane-shaped systems need a short-range
 * repulsion): U = c12/r^12 - c6/r^6 for r < rc, added to U2, F and W.
 * Cells are at least rc/2 wide and there must be >= 5 per axis (rc <= 2l/5);
 * a particle's candidates are the 125 cells around its own.  Within each cell
 * the members are ordered by index, so every sum has a fixed order and results
 * are bitwise reproducible. */
typedef struct rbe_real_ctx_s* rbe_real_ctx;

typedef struct {
  int64_t n;          /* particles, >= 1                                       */
  int32_t ntypes;     /* Lennard-Jones types, 0..64; 0 = Coulomb only          */
  int32_t precision;  /* RBE_PREC_FP64: pair arithmetic in FP64; RBE_PREC_FP32: */
                      /* in FP32 (separations formed in FP64, sums in FP64)    */
  double  alpha;      /* splitting parameter (the same alpha as rbe_config)    */
  double  rc;         /* cutoff, > 0                                           */
  double  coulomb;    /* Coulomb constant C, > 0                               */
} rbe_real_config;

/* Create a real-space context.
 *   d_q      : DEVICE, n charges (copied).
 *   d_type   : DEVICE, n int32 types in 0..ntypes-1 (copied), or NULL if ntypes = 0.
 *   h_lj     : HOST, ntypes*ntypes pairs (c12, c6), row-major over (t_i, t_j),
 *              symmetric, or NULL if ntypes = 0.
 *   box_host : HOST (lx, ly, lz); each >= 2.5 rc.  Cell storage is sized for
 *              sides up to 2x these values (at most 96 cells per axis).
 * Waits for the stream. */
rbe_status rbe_real_init(const rbe_real_config* cfg, const double* d_q, const int32_t* d_type,
                         const double* h_lj, const double* box_host, void* stream,
                         rbe_real_ctx* out);

/* Set the cell from host values (read now) for later evaluations. */
rbe_status rbe_real_set_box(rbe_real_ctx ctx, const double* box_host);

/* Read the cell from DEVICE memory (3 doubles) at every later evaluation.
 * A cell with a side below 2.5 rc, or beyond the capacity, is flagged on the
 * device (the grid is clamped) and reported by rbe_real_check. */
rbe_status rbe_real_set_box_dev(rbe_real_ctx ctx, const double* d_box);

/* Forces (written, or added when accumulate != 0), virial tensor (6 doubles,
 * xx yy zz xy xz yz; NULL to skip) and energy (1 double; NULL to skip) of the
 * real-space sum.  All arrays are DEVICE memory; positions may lie outside
 * the cell.  Asynchronous (five kernels on the context's stream; with
 * neighbour lists seven, of which the five that rebuild exit at once unless
 * the device decided to rebuild). */
rbe_status rbe_real_forces(rbe_real_ctx ctx, const double* d_x, const double* d_y,
                           const double* d_z, double* d_fx, double* d_fy, double* d_fz,
                           int accumulate, double* d_virial6, double* d_energy);

/* Neighbour lists (skin > 0; call once, before the first evaluation; waits):
 * each particle keeps the pairs closer than rc + skin at the last build, and
 * every evaluation tests them against rc with the minimum image; the lists
 * (and the cell list, now with cells at least (rc + skin)/2 wide) are rebuilt
 * on the device when 2 max|displacement since the build| + sqrt(3) max|cell
 * side change| >= skin (first evaluation: always).  The same pairs as without
 * lists, summed in the order of the list.  Needs every side >= 2.5 (rc +
 * skin) and n <= 2^25; a list holds 1.6 x the mean number of neighbours + 64
 * entries, at least 128 (a fuller one is flagged).  RBE_ERR_STATE if a skin is
 * set already. */
rbe_status rbe_real_set_skin(rbe_real_ctx ctx, double skin);

/* Wait; h_stats[0] = evaluations launched on the context, h_stats[1] =
 * neighbour-list builds among them (0 without a skin). */
rbe_status rbe_real_list_stats(rbe_real_ctx ctx, int64_t* h_stats);

/* Wait and report device-side flags: a cell below 2.5 x the search radius or
 * over capacity, a cell with more than 2048 members, or a neighbour list over
 * capacity (the evaluation is then incomplete). */
rbe_status rbe_real_check(rbe_real_ctx ctx);

/* Release the context (waits for the stream). */
void rbe_real_destroy(rbe_real_ctx ctx);

/* ---------------------------------------------------------------------------
 * Langevin NPT integrator (section 3.2 eq. (24), isotropic scaling of a
 * rectangular cell at its initial aspect ratio; appendix A eq.
 * (99999), semi-isotropic cell with gamma0 = 0; appendix A, rectangular cell
 * with anisotropic fluctuation: side lengths l_j with momenta p^l_j, driven
 * by V (P_jj - P)/l_j, eq. (e:instrectangular)), FP64, split as in section
 * 3.3:   B_V(h) B_R(h) A_V(h) A_R(h) O^p(dt) O(dt) A_R(h) A_V(h) | F, P | B_R(h) B_V(h)
 * with h = dt/2, every sub-flow solved exactly with the other variables
 * frozen:  A_R  r <- r e^{a h} + (p/m)(e^{a h} - 1)/a,
 *          B_R  p <- p e^{-a h} + F (1 - e^{-a h})/a,
 * a the per-axis scaling rate (V'/3V; or A'/2A, A'/2A, L'/L; or l_j'/l_j), the OU steps
 * exact (section 3.3), B_V driven by the instantaneous pressure tensor
 * (sum_i p_i p_i^T/m_i + W)/V of appendix C (iso: its trace/3; semi: (xx+yy)/2
 * against L, zz against A).  The B_V opening a step uses the pressure formed
 * at the end of the previous step (or by rbe_md_pressure before the first).
 * Noise: Philox4x64-10 keyed (seed, system_id), counter (step, i, 'nois', 0)
 * for particle i and (step, 0, 'cell', 0) for the cell; Box-Muller normals.
 * Units: forces and virials are multiplied by ftm to give mass x length /
 * time^2 (1 in reduced units; 4.184e-4 for kcal/mol/A with g/mol and fs);
 * kT and p_ext are in the force's energy units.  Momenta p = m v.
 * Positions, momenta and forces are caller-owned DEVICE arrays (SoA FP64). */
typedef struct rbe_md_ctx_s* rbe_md_ctx;

typedef struct {
  int64_t  n;            /* particles                                           */
  int32_t  box_mode;     /* RBE_BOX_ISO, RBE_BOX_SEMIISO or RBE_BOX_ANISO         */
  int32_t  reserved;     /* must be 0                                           */
  double   dt;           /* time step                                           */
  double   kT;           /* k_B T (energy units)                                */
  double   p_ext;        /* external pressure (energy / length^3)               */
  double   gamma_p;      /* particle friction (1/time), >= 0                     */
  double   gamma_cell;   /* cell friction (1/time), >= 0                         */
  double   mass_cell;    /* iso: mass M of V; semi: mass M_A of A; aniso: M_x    */
                         /* = M_y of l_x, l_y                                   */
  double   mass_cell_z;  /* semi: mass M_L of L; aniso: M_z (ignored for iso)   */
  double   ftm;          /* force units -> mass x length / time^2                */
  uint64_t seed;
  uint64_t system_id;
} rbe_md_config;

/* d_mass: DEVICE, n masses (copied).  box_host: initial cell (any aspect
 * ratio for iso, which keeps it; lx == ly for semi), momenta of the cell
 * start at 0.  Waits. */
rbe_status rbe_md_init(const rbe_md_config* cfg, const double* d_mass, const double* box_host,
                       void* stream, rbe_md_ctx* out);

/* Rigid 3-site molecules: atoms first + 3k (O), first + 3k + 1 and
 * first + 3k + 2 (H) for k < count, bonds O-H = d_oh and H-H = d_hh (the
 * positions must satisfy them, molecules whole, i.e. not split across the
 * periodic boundary); every molecule must have the masses of the first
 * (equal H masses).  Each position sub-flow is then followed by the
 * position constraint, solved in closed form per molecule (the result of
 * SHAKE: constraint forces along the old bonds), with the momentum change
 * the sub-flow's map gives it, and each momentum sub-flow by the projection
 * of the molecule's momenta onto rigid-body motions (the velocity stage of
 * RATTLE).  The pressure takes the molecular form
 *     P V = sum_free p p^T/m + sum_mol P P^T/M + W - sum_mol sum_a sym((r_a - R) F_a),
 * R, P the molecule's centre of mass and momentum.  count = 0 removes the
 * constraints.  Call before rbe_md_pressure; reads the masses (waits). */
rbe_status rbe_md_set_rigid(rbe_md_ctx ctx, int64_t first, int64_t count, double d_oh,
                            double d_hh);

/* Instantaneous pressure from the current state and the virial tensors (6
 * doubles each, DEVICE, either may be NULL), without moving anything: call
 * once before the first step.  With rigid molecules it also projects their
 * momenta (stored back) and needs positions and forces.  Asynchronous. */
rbe_status rbe_md_pressure(rbe_md_ctx ctx, const double* d_x, const double* d_y,
                           const double* d_z, double* d_px, double* d_py, double* d_pz,
                           const double* d_fx, const double* d_fy, const double* d_fz,
                           const double* d_virial_k, const double* d_virial_r);

/* B_V B_R A_V A_R O^p O A_R A_V of step `step` on positions and momenta with
 * the forces of the previous evaluation.  Afterwards rbe_md_box_dev() holds
 * the cell for this step's force evaluation.  Asynchronous. */
rbe_status rbe_md_first_half(rbe_md_ctx ctx, uint64_t step, double* d_x, double* d_y,
                             double* d_z, double* d_px, double* d_py, double* d_pz,
                             const double* d_fx, const double* d_fy, const double* d_fz);

/* B_R with the new forces (and the momentum projection of rigid molecules,
 * which needs the positions), the pressure tensor from the momenta and the
 * virial tensors (DEVICE, 6 doubles each, either may be NULL), then B_V.
 * Asynchronous. */
rbe_status rbe_md_second_half(rbe_md_ctx ctx, const double* d_x, const double* d_y,
                              const double* d_z, double* d_px, double* d_py, double* d_pz,
                              const double* d_fx, const double* d_fy, const double* d_fz,
                              const double* d_virial_k, const double* d_virial_r);

/* DEVICE pointer to the 3 side lengths of the current step's cell (valid
 * after rbe_md_first_half; feed it to rbe_rescale_box_dev / rbe_real_set_box_dev). */
const double* rbe_md_box_dev(rbe_md_ctx ctx);

/* Waits; h_state[32] = lx ly lz, volume, pV, pA, pL, pressure tensor (6,
 * energy/length^3), kinetic tensor sum p p^T/m (6, energy; rigid molecules
 * contribute P P^T/M), error flags, step, A, L, V, the rigid-molecule
 * correction sum sym((r - R) F) (6, energy), rigid molecules, 0.  In the
 * anisotropic mode entries 4-6 hold the momenta of l_x, l_y, l_z. */
rbe_status rbe_md_get_state(rbe_md_ctx ctx, double* h_state);

/* Waits; RBE_ERR_STATE if the cell collapsed or became non-finite, or a
 * rigid-molecule position constraint had no solution (flags cleared). */
rbe_status rbe_md_check(rbe_md_ctx ctx);

void rbe_md_destroy(rbe_md_ctx ctx);

/* ---------------------------------------------------------------------------
 * Served batching: many independent NPT systems, each the full step above
 * (Fourier part, real-space pairs, integrator) with its own state kept on
 * the device between steps, advanced together.  Admission is bounded by a
 * device-memory budget and a slot count.  A fused step launches each kernel
 * of the step once for all admitted systems (a system's blocks are its own
 * launch plan's blocks, so its arithmetic and reduction order are those it
 * has alone: results do not depend on which other systems share the step).
 * All calls on one batch must come from one host thread. */
typedef struct rbe_batch_s* rbe_batch;

typedef struct {
  int32_t  precision;    /* rbe_precision of the Fourier part, every system  */
  int32_t  max_systems;  /* slots, 1..4096                                     */
  int64_t  hbm_budget;   /* device bytes the admitted systems may hold (> 0)    */
  int32_t  real_precision; /* rbe_precision of the real-space pair arithmetic */
  int32_t  reserved;     /* must be 0                                          */
} rbe_batch_config;

typedef struct {
  int64_t  n;            /* particles                                          */
  int32_t  p;            /* frequencies per step (batch size P)                */
  int32_t  ntypes;       /* Lennard-Jones types (0: none)                      */
  int32_t  box_mode;     /* RBE_BOX_ISO (any aspect ratio, kept),              */
                         /* RBE_BOX_SEMIISO or RBE_BOX_ANISO                    */
  int32_t  sampler;      /* rbe_sampler of the Fourier part (RBE_SAMPLER_MH:    */
                         /* one chain move per step, as rbe_set_sampler)        */
  double   alpha;        /* Ewald splitting parameter (length^-2)              */
  double   coulomb;      /* Coulomb constant in the force units                */
  double   rc;           /* real-space cutoff                                  */
  double   dt, kT, p_ext, gamma_p, gamma_cell, mass_cell, mass_cell_z, ftm;
                         /* integrator parameters, as in rbe_md_config         */
  uint64_t seed;         /* Philox key word 0                                  */
  uint64_t system_id;    /* Philox key word 1 (e.g. the request id)            */
  int64_t  rigid_first;  /* rigid 3-site molecules as rbe_md_set_rigid         */
  int64_t  rigid_count;  /* (0: none)                                          */
  double   d_oh, d_hh;   /* their bond lengths                                 */
  double   skin;         /* real-space neighbour-list skin (0: none), as       */
                         /* rbe_real_set_skin                                  */
} rbe_system_desc;

/* stream: hipStream_t for every launch and copy of the batch (NULL: the null
 * stream).  Allocates two pinned argument-table buffers. */
rbe_status rbe_batch_create(const rbe_batch_config* cfg, void* stream, rbe_batch* out);

/* Device bytes a system holds while admitted (its state arrays and the
 * buffers of its three contexts, each rounded up to 256 bytes): the figure
 * admission charges against the budget. */
rbe_status rbe_batch_footprint(const rbe_system_desc* desc, const double* box_host,
                               int64_t* bytes);

/* Admit one system.  HOST arrays: h_pos [n][3], h_mom [n][3] (NULL: zero
 * momenta), h_q [n] (neutral), h_mass [n], h_type [n] and h_lj
 * [ntypes][ntypes][2] = (c12, c6) when ntypes > 0; box_host [3].  Copies
 * everything to the device, evaluates the opening forces and pressure (the
 * Fourier batch of step 2^63) and waits.  RBE_ERR_CAPACITY, with nothing
 * allocated, when no slot is free or the footprint would take the batch
 * over its budget; *slot gets the slot index (>= 0) on success. */
rbe_status rbe_batch_admit(rbe_batch b, const rbe_system_desc* desc, const double* h_pos,
                           const double* h_mom, const double* h_q, const double* h_mass,
                           const int32_t* h_type, const double* h_lj, const double* box_host,
                           int32_t* slot);

/* One NPT step of every admitted system (each at its own step index, which
 * then advances).  fused = 1: every kernel launched once for all systems,
 * the argument tables copied in one transfer; fused = 0: each system's
 * kernels launched on their own, one system after another (the same
 * arithmetic).  Asynchronous.  A step that fails after some systems' host
 * state has advanced (an argument-table overflow, a launch error) leaves
 * the batch refusing every later step with RBE_ERR_STATE: release or
 * destroy it. */
rbe_status rbe_batch_step(rbe_batch b, int32_t fused);

/* The Fourier-space step alone for every admitted system (a1-a6: cell
 * tables, the batch of the system's current step, rho, forces, virial and
 * energy, section 4.2 eq. (appforce), (apppress)) at its current positions
 * and cell: forces overwrite the system's force arrays; positions, momenta
 * and cell stay; the step counter advances.  fused as rbe_batch_step (one
 * launch per kernel shape for all systems, or per-system launches).  Not to
 * be mixed with rbe_batch_step on the same systems (a full step would start
 * from Fourier-only forces).  Asynchronous. */
rbe_status rbe_batch_step_fourier(rbe_batch b, int32_t fused);

/* Waits for the batch's stream. */
rbe_status rbe_batch_sync(rbe_batch b);

/* Waits; h_stats[2] = the slot's real-space evaluations and neighbour-list
 * builds so far, as rbe_real_list_stats. */
rbe_status rbe_batch_list_stats(rbe_batch b, int32_t slot, int64_t* h_stats);

/* Waits; h_pos, h_mom, h_frc [n][3]: positions, momenta and the forces of
 * the last evaluation (each may be NULL); h_state [32] as rbe_md_get_state
 * (may be NULL). */
rbe_status rbe_batch_read(rbe_batch b, int32_t slot, double* h_pos, double* h_mom,
                          double* h_frc, double* h_state);

/* Waits; the device-side error flags of the slot's three contexts. */
rbe_status rbe_batch_check(rbe_batch b, int32_t slot);

/* Steps the slot's system has taken since admission. */
rbe_status rbe_batch_slot_step(rbe_batch b, int32_t slot, int64_t* step);

/* Waits for launched work, frees the slot and returns its bytes to the budget. */
rbe_status rbe_batch_release(rbe_batch b, int32_t slot);

/* h[4] = admitted systems, bytes held, budget, steps launched. */
rbe_status rbe_batch_info(rbe_batch b, int64_t* h);

/* Kernel timing of the next max_steps fused steps (0: off; waits): HIP events
 * on the batch's stream before and after each kernel family. */
rbe_status rbe_batch_timing_enable(rbe_batch b, int32_t max_steps);

/* Waits; h_ms[5] = summed device time (ms) of the integrator's first half,
 * the structure factors, the forces, the real-space kernels and the
 * integrator's second half over the timed steps; *h_steps their number;
 * *h_np the summed N p (Fourier pairs) of those steps.  Resets the count. */
rbe_status rbe_batch_timing_read(rbe_batch b, double* h_ms, int32_t* h_steps, double* h_np);

void rbe_batch_destroy(rbe_batch b);

/* Text of the last error reported to the calling thread ("" if none). */
const char* rbe_last_error(void);

/* Library version string. */
const char* rbe_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RBE_H */
