/*
 * ewald.h -- C ABI of libewald.so: batched periodic Ewald energies and
 * single-electron move deltas for quantum Monte Carlo walkers on one MI355X.
 *
 * The operation is the periodic Coulomb energy of the paper's Sec. 2.2
 * ("Ewald summation", Eqs. (2)-(6)): for charges q_i at r_i in a periodic
 * cell with lattice vectors a_i (rows of `lattice`) and split parameter
 * alpha = sqrt(gamma),
 *
 *   E = E_real + E_recip + E_self + E_background
 *   E_real       = sum_{i<j} q_i q_j erfc(alpha r_ij)/r_ij over the minimum image,
 *                  kept iff r_ij < r_cut (r_cut <= r_inscribed, so at most one
 *                  image of each pair contributes and no particle sees its own
 *                  images)
 *   E_recip      = sum_{G in H} w(|G|) |rho(G)|^2,  rho(G) = sum_i q_i exp(i G.r_i)
 *                  w = (4 pi/Omega) exp(-G^2/4alpha^2)/G^2        (3D, Eqs. (3)-(4))
 *                  w = (2 pi/A) erfc(G/2alpha)/G                  (2D, z = 0, Eqs. (5)-(6))
 *                  H = one of each pair +-G with 0 < |G| <= g_cut (a G whose first
 *                  nonzero reduced coordinate is positive), which is why w
 *                  carries a factor 2
 *   E_self       = -(alpha/sqrt(pi)) sum_i q_i^2
 *   E_background = -(pi/(2 Omega alpha^2)) Q^2 (3D),  -(sqrt(pi)/(A alpha)) Q^2 (2D)
 *
 * Layered 2D systems (two planes at heights z_0, z_1, d = z_1 - z_0; the
 * z-dependent terms of Eq. (5)): rho_l(G) per plane,
 *   E_recip = sum_{G in H} [w (|rho_0|^2 + |rho_1|^2) + 2 w_x Re(rho_0 conj(rho_1))],
 *   w_x = (pi/A) [e^{dG} erfc(G/2alpha + d alpha) + e^{-dG} erfc(G/2alpha - d alpha)]/G,
 * real-space pairs of different planes at distance sqrt(r^2 + d^2), and
 *   E_background = 1/2 sum_{l,m} Q_l Q_m c(z_l - z_m),
 *   c(z) = -(2 pi/A) [z erf(z alpha) + exp(-alpha^2 z^2)/(alpha sqrt(pi))].
 *
 * and, optionally, the Jastrow value of Sec. 2.3: the long-range plane-wave
 * term (Eq. (9) expressed through the same structure factor) plus, when the
 * system has one, the two-body polynomial term u of Eq. (8)
 *
 *   J = sum_{G in H} a_{s(G)} |rho(G)|^2 + sum_{i<j mobile} u_{c(i,j)}(r_ij),
 *   s(G) = shell of equal |G|, ascending.
 *
 * A single-particle move (Sec. 2.1: propose a move of one particle, decide,
 * update) changes particle k from r_k to r'; the library returns
 *   dE = q_k sum_{j != k} q_j [phi(r' - r_j) - phi(r_k - r_j)]
 *        + sum_H w [2 Re(conj(rho) delta) + |delta|^2],
 *   delta(G) = q_k (exp(iG.r') - exp(iG.r_k)),   phi(r) = erfc(alpha r)/r,
 * (and dJ with a_s in place of w) and, when the move is accepted, updates
 * rho <- rho + delta and r_k <- r'.
 *
 * Precision forms (Sec. 6.1: set-up tables always in double precision):
 *   EWALD_FP64        every step in FP64.
 *   EWALD_FP32_MIXED  move deltas: phases exp(2 pi i frac(n.s)) in FP32 from
 *                     FP64 fractional coordinates, the erf part of phi in FP32,
 *                     FP32 partial sums with Kahan compensation; geometry
 *                     (displacement, minimum image, r^2, 1/r), constants and
 *                     the running rho in FP64, and rho rebuilt from the
 *                     positions in FP64 every `refresh_every` accepted moves.
 *                     Energies (ewald_energy_batch) are computed in FP64 as in
 *                     the FP64 form: they add ~N^2/4 pair terms of one sign,
 *                     where an FP32 bias of the pair function would add up.
 *
 * Conventions
 *   - Units: Hartree atomic units (bohr, Hartree).
 *   - Ownership: ewald_setup copies every host input; the caller may free them
 *     on return.  Device tables are owned by the ewald_sys / ewald_batch and
 *     freed by the matching _destroy.  Every per-walker buffer (positions,
 *     state, proposals, outputs) is caller-owned DEVICE memory.
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = default
 *     stream).  Batch calls only enqueue kernels: they never allocate, copy
 *     to the host or synchronise, so they can be captured in a HIP graph.
 *   - Errors: arguments are validated synchronously before anything is
 *     enqueued; a non-OK status means nothing was enqueued and
 *     ewald_last_error() (thread-local) holds a message.  No C++ exception
 *     crosses the ABI.  Faults inside kernels surface at the caller's next
 *     synchronisation.  A move index k outside [0, n_mobile) is not an error
 *     status (it is device data): that walker's delta is NaN and no move is
 *     pending for it.  Coincident particles or NaN positions give non-finite
 *     results.
 *   - Thread safety: ewald_sys and ewald_batch are immutable after creation
 *     except for the host-side state-phase bookkeeping of each batch (which
 *     is locked); concurrent calls on distinct state buffers are safe.
 */
#ifndef EWALD_H
#define EWALD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ewald_sys ewald_sys;     /* one periodic cell, its charges and G tables */
typedef struct ewald_batch ewald_batch; /* walker -> system map, packed layout        */

typedef enum {
    EWALD_OK = 0,
    EWALD_E_ARG = 1,     /* bad argument (null pointer, count, mixed batch, ...) */
    EWALD_E_RCUT = 2,    /* r_cut <= 0 or r_cut > r_inscribed                    */
    EWALD_E_GCUT = 3,    /* g_cut <= 0, or the G set exceeds the library limits  */
    EWALD_E_LATTICE = 4, /* singular or non-finite lattice                       */
    EWALD_E_NOMEM = 5,   /* host or device allocation failed                     */
    EWALD_E_HIP = 6,     /* a HIP runtime call failed (no device, launch error)  */
    EWALD_E_STATE = 7    /* call order: move before energy, accept w/o pending   */
} ewald_status;

typedef enum { EWALD_FP64 = 0, EWALD_FP32_MIXED = 1 } ewald_precision;

/* Library limits (checked by ewald_setup). */
#define EWALD_MAX_PARTICLES 2048 /* n_mobile + n_fixed per system               */
#define EWALD_MAX_NRED 120       /* largest |n_d| of a G vector in reduced units */
#define EWALD_MAX_SEGMENTS 2048  /* G segments (4 G each) per system             */

typedef struct {
    int dim;                   /* 2 or 3                                               */
    double lattice[3][3];      /* rows a_i in bohr; a 2D cell uses lattice[0..1][0..1] */
    int n_fixed;               /* fixed ions (>= 0)                                    */
    const double *fixed_pos;   /* host [n_fixed][dim] Cartesian bohr                   */
    const double *fixed_q;     /* host [n_fixed]                                       */
    int n_mobile;              /* mobile particles (electrons), >= 1                   */
    const double *mobile_q;    /* host [n_mobile]                                      */
    double alpha;              /* Ewald split parameter, 1/bohr, > 0                   */
    double g_cut;              /* |G| <= g_cut (inclusive, relative slack 1e-12 on G^2)*/
    double r_cut;              /* real-space cutoff, 0 < r_cut <= r_inscribed          */
    ewald_precision precision;
    int refresh_every;         /* K: rho rebuilt in FP64 every K accepted moves of a   */
                               /* walker in the FP32-mixed form; 0 = never             */
    int n_jastrow;             /* number of shell coefficients a_s (0: no Jastrow);    */
                               /* coefficients past the last shell are ignored         */
    const double *jastrow_a;   /* host [n_jastrow]                                     */
    /* Optional Jastrow two-body polynomial term (Sec. 2.3, Eq. (8)) over pairs  */
    /* of mobile particles at their minimum-image distance r:                     */
    /*   u_c(r) = sum_{l < u_terms} u_alpha[c][l] r^l (r - u_cutoff)^u_C, r < L_u  */
    /* c = 0 for equal spin labels, 1 for unequal ones (parallel and antiparallel */
    /* spins); the fixed ions take no part.                                       */
    int u_terms;               /* N_u + 1 coefficients per channel (0: no u term);     */
                               /* u_terms - 1 + u_C <= 15                               */
    int u_C;                   /* C >= 1                                               */
    double u_cutoff;           /* L_u, 0 < L_u <= r_inscribed                          */
    const double *u_alpha;     /* host [2][u_terms]                                    */
    const int32_t *mobile_spin; /* host [n_mobile] labels 0 or 1 (NULL: all 0)        */
    /* Optional layered two-dimensional system (dim = 2; Sec. 2.2, Eq. (5) with  */
    /* z != 0): particles in two parallel planes at heights layer_z[0..1];       */
    /* moves stay in their plane.  Not combined with Jastrow terms.              */
    int n_layers;              /* 0 or 1: one plane (z = 0); 2: two planes             */
    double layer_z[2];         /* heights of the planes (bohr)                         */
    int n_mobile_layer0;       /* mobile particles 0..n0-1 lie in plane 0, the rest    */
                               /* in plane 1                                           */
    const int32_t *fixed_layer; /* host [n_fixed] plane (0/1) of each ion (NULL: 0)    */
} ewald_sys_desc;

/* Build the cell's tables on the host in FP64 (reciprocal lattice, G set,
 * shells, weights, fixed-ion structure factor, constants, minimum-image
 * candidates): the quantities of Sec. 2.2, Eqs. (2)-(6), that depend on the
 * cell alone, set up once and kept in double precision (Sec. 6.1).  Touches
 * no device; device copies are made by ewald_batch_create.  Status: E_ARG,
 * E_LATTICE, E_RCUT, E_GCUT, E_NOMEM. */
ewald_status ewald_setup(const ewald_sys_desc *desc, ewald_sys **out);

/* Sizes and constants of a system.  Any output pointer may be NULL.
 * n_g: |H|; n_slots: stored G slots including padding (4 per segment);
 * e_const = E_self + E_background + the fixed-ion real-space pair energy. */
ewald_status ewald_sys_query(const ewald_sys *sys, int *n_g, int *n_slots, int *n_shells,
                             double *r_inscribed, double *e_const);

/* Host copies of the per-slot tables in the library's storage order (the
 * order of rho in the walker state).  For each slot: reduced coordinates
 * n[slot][3] (G = sum_d n_d b_d), weight w, Jastrow coefficient, shell index
 * (-1 for padding slots, whose weights are 0).  Arrays hold n_slots entries;
 * any pointer may be NULL. */
ewald_status ewald_sys_tables(const ewald_sys *sys, int32_t *n, double *weight, double *jastrow,
                              int32_t *shell);

/* Minimum-image candidate lattice offsets (one of each +-pair), Cartesian
 * [n][3]; `cand` may be NULL to query the count. */
ewald_status ewald_sys_candidates(const ewald_sys *sys, int *n_cand, double *cand);

/* The minimum-image geometry the kernels use for this cell.  If the lattice
 * contains mutually orthogonal vectors spanning a sublattice of index m <= 2
 * whose nonzero coset is offset by half box sides (simple-cubic, bcc, fcc and
 * hexagonal cells), *index = m and box[0..dim) receives their lengths
 * (bohr): pair distances are then reduced per axis in that box with one
 * extra image check for the coset.  Otherwise *index = 0 and the general
 * reduction (fractional rint plus the candidate offsets above) is used.
 * Either pointer may be NULL; box must hold 3 doubles.  Status: E_ARG. */
ewald_status ewald_sys_geometry(const ewald_sys *sys, int *index, double *box);

void ewald_sys_destroy(ewald_sys *sys);

/* A batch of n_walkers walkers; walker w belongs to sys[walker_sys[w]]
 * (host array).  All systems must share dim and precision.  Copies the
 * systems' tables to the current HIP device (once per system).  The systems
 * must outlive the batch.  Status: E_ARG, E_NOMEM, E_HIP. */
ewald_status ewald_batch_create(ewald_sys *const *sys, int n_sys, const int *walker_sys,
                                int n_walkers, ewald_batch **out);

/* Packed layout.  pos_offsets (host [n_walkers + 1], may be NULL): walker w's
 * mobile positions are rows pos_offsets[w] .. pos_offsets[w+1]-1 of a
 * [total][dim] FP64 array.  *state_bytes: size of the device state buffer
 * (256-byte aligned). */
ewald_status ewald_batch_layout(const ewald_batch *b, size_t *pos_offsets, size_t *state_bytes);

/* Byte offsets, inside the state buffer, of walker w's header, wrapped
 * fractional positions ([n_mobile][dim] FP64) and rho ([n_slots] complex
 * FP64, (re, im) pairs, slot order of ewald_sys_tables). Header layout:
 * int32 counter (accepted moves since the last rho rebuild), int32 pending_k
 * (-1: none), int32 n_accepts, int32 n_refresh, double pending_s[3], double
 * drift_max (largest |rho_running - rho_rebuilt| seen at a rebuild). */
ewald_status ewald_state_offsets(const ewald_batch *b, int walker, size_t *hdr, size_t *pos,
                                 size_t *rho);

void ewald_batch_destroy(ewald_batch *b);

/* Energies of all walkers (Sec. 2.2, Eqs. (2)-(6)).
 *   pos      device [total][dim] Cartesian positions (ewald_batch_layout order)
 *   state    device, ewald_batch_layout bytes; (re)initialised: wrapped
 *            positions, rho in FP64, counters zeroed, no pending move
 *   energy   device [n_walkers] out
 *   jastrow  device [n_walkers] out, or NULL */
ewald_status ewald_energy_batch(ewald_batch *b, const double *pos, void *state, double *energy,
                                double *jastrow, void *stream);

/* Energy change of one proposed single-particle move per walker (Sec. 2.1).
 *   k        device [n_walkers] index of the moved particle in [0, n_mobile)
 *   new_pos  device [n_walkers][dim] Cartesian proposal (any periodic image)
 *   delta    device [n_walkers] out, E(new) - E(old)
 *   djastrow device [n_walkers] out, J(new) - J(old), or NULL
 * Records the move as pending in the state (replacing an earlier pending
 * move); rho and positions are unchanged.  E_STATE before ewald_energy_batch
 * on this state buffer. */
ewald_status ewald_move_delta_batch(ewald_batch *b, void *state, const int32_t *k,
                                    const double *new_pos, double *delta, double *djastrow,
                                    void *stream);

/* The update step of a single-particle move (Sec. 2.1: after the accept/reject
 * decision the configuration and its cached quantities are updated).
 * Apply (accept[w] != 0) or drop (accept[w] == 0) each walker's pending move:
 * rho <- rho + delta in FP64, r_k <- r', counters; in the FP32-mixed form a
 * walker reaching refresh_every accepted moves gets rho rebuilt from its
 * positions in FP64.  E_STATE if no move is pending. */
ewald_status ewald_accept_batch(ewald_batch *b, void *state, const uint8_t *accept, void *stream);

/* One step of the single-particle move loop (Sec. 2.1): the accept/reject
 * decision on the move left pending by the previous call, then the energy
 * change of the next proposed move.  Same results and state as
 *   ewald_accept_batch(accept_prev) followed by
 *   ewald_move_delta_grad_batch(k, new_pos, delta, djastrow, jgrad, jlap),
 * with the accept's update of rho (rho <- rho + delta in FP64) applied while
 * the delta streams rho, so that rho is read once per step rather than
 * twice for an accepted move.
 *   accept_prev  device [n_walkers], or NULL: no decision to apply (exactly
 *                ewald_move_delta_grad_batch); non-NULL needs a pending move
 *                (E_STATE otherwise), as ewald_accept_batch does
 *   k, new_pos, delta, djastrow, jgrad, jlap: as ewald_move_delta_grad_batch
 * The new move is left pending.  In the FP32-mixed form a walker whose accept
 * reaches refresh_every accepted moves gets rho rebuilt in FP64 before its
 * delta is taken, as in the two-call sequence (a second, short launch).
 * Status as for ewald_move_delta_grad_batch. */
ewald_status ewald_step_batch(ewald_batch *b, void *state, const uint8_t *accept_prev, const int32_t *k,
                              const double *new_pos, double *delta, double *djastrow, double *jgrad,
                              double *jlap, void *stream);

/* n_steps consecutive proposals per walker in one launch, rho kept on chip: a
 * sequence of the single-particle moves of Sec. 2.1, each with its energy
 * change as defined for ewald_move_delta_batch (Sec. 2.2, Eqs. (2)-(6)).
 * Same results as n_steps pairs of ewald_move_delta_batch + ewald_accept_batch
 * (accept decisions must therefore be known in advance, as when the Ewald
 * energy is evaluated after a sweep of moves).
 *   k [n_steps][n_walkers], new_pos [n_steps][n_walkers][dim],
 *   accept [n_steps][n_walkers], delta/djastrow [n_steps][n_walkers] (djastrow
 *   may be NULL); all device.  E_STATE before ewald_energy_batch. */
ewald_status ewald_run_moves_batch(ewald_batch *b, void *state, int n_steps, const int32_t *k,
                                   const double *new_pos, const uint8_t *accept, double *delta,
                                   double *djastrow, void *stream);

/* Jastrow derivatives (Sec. 2.3, Eq. (9); the values and derivatives of the
 * p term are what Sec. 5.2 offloads, and the kinetic energy and drift of QMC
 * need the gradient and the Laplacian, Sec. 2.1).  The same calls as
 * ewald_move_delta_batch and ewald_run_moves_batch, which also return, for
 * each proposed move of particle k to r', the gradient and the Laplacian of
 * J with respect to r_k at the proposed configuration (particle k at r',
 * whether or not the move is then accepted):
 *   grad_k J = -2 q_k sum_{G in H} a_s(G) G Im(conj(rho') exp(iG.r'))
 *   lap_k J  = -2 q_k sum_{G in H} a_s(G) |G|^2 [Re(conj(rho') exp(iG.r')) - q_k]
 *   rho' = rho + q_k (exp(iG.r') - exp(iG.r_k))
 * (for unit charges these are the derivatives of 2 sum_{j != k} p(r_k - r_j)),
 * plus, with a u term (Eq. (8)), over the mobile j != k with r = |d| < L_u,
 * d the minimum-image displacement r' - r_j:
 *   grad_k U = sum_j u'(r) d / r,   lap_k U = sum_j [u''(r) + (dim - 1) u'(r) / r].
 * The u term is evaluated in FP64 in both precision forms.
 *   jgrad  device out, Cartesian: [n_walkers][dim] (move_delta) or
 *          [n_steps][n_walkers][dim] (run_moves)
 *   jlap   device out: [n_walkers] or [n_steps][n_walkers]
 * Both NULL: exactly ewald_move_delta_batch / ewald_run_moves_batch.  An
 * invalid k gives NaN derivatives.  Status as for those calls, plus E_ARG if
 * only one of jgrad/jlap is given or the batch has neither Jastrow
 * coefficients nor a u term.
 * The FP32-mixed form computes z = conj(rho') exp(iG.r') in FP32 and sums
 * in FP64 across segments. */
ewald_status ewald_move_delta_grad_batch(ewald_batch *b, void *state, const int32_t *k,
                                         const double *new_pos, double *delta, double *djastrow,
                                         double *jgrad, double *jlap, void *stream);
ewald_status ewald_run_moves_grad_batch(ewald_batch *b, void *state, int n_steps, const int32_t *k,
                                        const double *new_pos, const uint8_t *accept, double *delta,
                                        double *djastrow, double *jgrad, double *jlap, void *stream);

/* Launch shape of ewald_run_moves_batch (the batching of Sec. 5.1; the paper
 * tunes gang and vector sizes by hand, Sec. 3.3).  One workgroup serves one walker;
 *   threads        workgroup size, which fixes segments of 4 G per thread and
 *                  particles per thread: 0 = default for the largest segment
 *                  count s of the batch (s <= 512: 256; s <= 1024: 1024;
 *                  s <= 2048: 512); also available: 1024 for s <= 1024
 *                  and 512 for 512 < s <= 1024; other values give E_ARG
 *   chunk          at most this many moves staged per chunk, 1..64 (fewer
 *                  when LDS does not hold them), or 0 = as many as LDS allows
 *                  without lowering the workgroups per CU
 *   general_frame  1 = the general minimum-image reduction even when the
 *                  cell has an orthogonal-sublattice frame (ewald_sys_geometry);
 *                  applies to ewald_energy_batch as well
 *   waves          waves per SIMD the kernel is compiled for, for workgroups
 *                  of 256 and 512 threads: 0 or 2 = default (256 registers
 *                  per lane, constants in vector registers), 3 or 4 = more
 *                  workgroups per CU with the constants in scalar registers
 *                  (256 threads: 3 or 4; 512 threads with 2 segments per
 *                  thread: 4); other combinations give E_ARG (1024-thread
 *                  workgroups run at four waves per SIMD by construction).
 *                  The Jastrow-derivative sweep (ewald_run_moves_grad_batch)
 *                  runs 512 x 2 at two waves whatever this says
 *   walkers_per_block  0 = one workgroup per walker, dispatched by the
 *                  hardware in the batch's launch order (most expensive
 *                  walker first); W > 0 = ceil(n_walkers / W) workgroups,
 *                  each taking the next walker, in the same order, from a
 *                  work counter until all are done (the counter is the int32
 *                  at byte 192 of the state buffer, inside the first walker's
 *                  header; it is reset by a kernel launched on the stream
 *                  before the sweep, so such calls stay graph-capturable);
 *                  E_ARG if negative, or if > 0 with waves 3 or 4 (the
 *                  queue-mode kernels are compiled for two waves per SIMD)
 * Results do not depend on the choice beyond rounding order (the queue mode
 * computes each walker exactly as one workgroup per walker does).  Not to be
 * called concurrently with launches on the same batch. */
ewald_status ewald_batch_set_tuning(ewald_batch *b, int threads, int chunk, int general_frame, int waves,
                                    int walkers_per_block);

/* The launch shape ewald_run_moves_batch will use: workgroup size, moves per
 * chunk, frame (1 = general), fused = 0 when the walkers do not fit the
 * fused kernel's LDS layout (then it runs the per-step
 * kernels in turn), and the waves per SIMD a 256- or 512-thread kernel is
 * compiled for (0 for 1024 threads and when not fused), and the walkers
 * per workgroup (0: one workgroup per walker, and when not fused), so that
 * the values can be passed back to ewald_batch_set_tuning.
 * Any output pointer may be NULL. */
ewald_status ewald_batch_get_tuning(ewald_batch *b, int *threads, int *chunk, int *general_frame,
                                    int *fused, int *waves, int *walkers_per_block);

/* The launch-shape choice that Sec. 3.3 makes by hand for each GPU (gang and
 * vector sizes), made by measurement: time every launch shape of
 * ewald_run_moves_batch on this batch and keep the fastest
 * (ewald_batch_set_tuning); shapes within 8 % of the fastest
 * are timed twice more, interleaved, and compared by their best time; then
 * the queue mode of ewald_batch_set_tuning (walkers_per_block 1, and the
 * count that leaves as many workgroups as that shape fits on the device at
 * once) is timed against one workgroup per walker, interleaved.  The
 * probe runs n_moves (1..4096)
 * proposals per walker, every other one accepted, on a device copy of
 * `state`, which must be ready (after ewald_energy_batch, no pending move)
 * and is left unchanged; in the FP32-mixed form n_moves >= 2 refresh_every
 * makes the probe include rho rebuilds.  With a
 * cache_path, a tuning stored there for the same device architecture and
 * batch shape is applied without timing (one that ewald_batch_set_tuning
 * rejects is measured afresh), and a new one is appended (one text line per
 * shape; the last line for a shape wins).  Allocates temporary device buffers and synchronises
 * `stream`: a set-up call, not for graph capture.  Status: E_ARG, E_STATE,
 * E_HIP. */
ewald_status ewald_autotune(ewald_batch *b, void *state, int n_moves, const char *cache_path,
                            void *stream);

/* ---- Blip orbitals (Sec. 2.4) ------------------------------------------------
 * Orbitals re-represented on a periodic grid of n1 x n2 x n3 points along the
 * lattice vectors.  With fractional coordinates s = r A^-1 and x_d = n_d s_d,
 *   psi_m(r) = sum_{i,j,k} a[i][j][k][m] Th(x_1 - i) Th(x_2 - j) Th(x_3 - k)
 * (grid indices periodic), with the cubic B-spline blip function
 *   Th(x) = 1 - 3/2 x^2 + 3/4 |x|^3 (|x| <= 1),  1/4 (2 - |x|)^3 (1 < |x| < 2),
 * zero beyond, so 4 x 4 x 4 grid points take part at each point.  The
 * evaluation after a move (the paper's 64-element products of blip functions
 * with each orbital's coefficients, Sec. 5.3) is batched over many points. */
typedef struct ewald_blip ewald_blip;

/* A grid over the cell with rows a_i = lattice[i] (3D, bohr), grid[d] in
 * [4, 4096] points along a_d, n_orb >= 1 orbitals.  Host only; the handle
 * holds no device memory.  Status: E_ARG, E_LATTICE, E_NOMEM. */
ewald_status ewald_blip_create(const double lattice[3][3], const int grid[3], int n_orb, ewald_blip **out);
void ewald_blip_destroy(ewald_blip *b);

/* Orbitals at n_points Cartesian points (any position; wrapped into the cell):
 *   coef  device [n1][n2][n3][n_orb] FP64, caller-owned (orbital index
 *         fastest; 16-byte aligned with even n_orb for the paired loads)
 *   pos   device [n_points][3]
 *   val   device out [n_points][n_orb]
 *   grad  device out [n_points][3][n_orb] (Cartesian), or NULL
 *   lap   device out [n_points][n_orb], or NULL (both or neither)
 * FP64 throughout.  Enqueues one kernel on `stream`; no allocation, no
 * synchronisation (graph-capturable).  Status: E_ARG, E_HIP. */
ewald_status ewald_blip_eval_batch(const ewald_blip *b, const double *coef, int n_points, const double *pos,
                                   double *val, double *grad, double *lap, void *stream);

/* Per-call timers (the role of the paper's subroutine timers, Sec. 3.2:
 * invocations and times per activity, reported at the end of a run).  When
 * on, every call that enqueues GPU work (ewald_energy_batch, the move-delta,
 * accept, step and run-moves calls, ewald_autotune, ewald_blip_eval_batch)
 * counts an invocation, its host time, and the GPU time between two events
 * recorded on its stream around the work it enqueues (not recorded while the
 * stream is being captured into a graph).  The events are read only when a
 * report is made, so timing adds no synchronisation to the calls.  Initially
 * on iff the environment variable EWALD_TIMING is set to a value other than
 * "0"; process-wide.
 *   ewald_timing_enable: on (!= 0) or off; always EWALD_OK
 *   ewald_timing_report: waits for the recorded events, then writes one
 *     header line and one line per call name,
 *       "<call> <calls> <gpu_calls> <gpu_ms_total> <gpu_ms_mean> <host_ms_total>",
 *     NUL-terminated, into buf (len bytes, caller-owned); reset != 0 clears
 *     the counts afterwards.  E_ARG if buf is NULL with len > 0, or if the
 *     report did not fit (it is then truncated). */
ewald_status ewald_timing_enable(int on);
ewald_status ewald_timing_report(char *buf, size_t len, int reset);

/* Thread-local message for the last non-OK status of this thread. */
const char *ewald_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EWALD_H */
