/*
 * kbe.h -- C ABI of the MI355X (gfx950) Kadanoff-Baym propagation library.
 *
 * The library advances the two-time lesser/greater Green's functions
 * G^{<,>}_{ab}(k; t, t') of a lattice model, one time slice per step, exactly as
 * arXiv 2505.19467 states the problem: Algorithm "prop" (predictor, corrector
 * passes, re-evaluation), eq. (Green) for the per-k equations of motion, eq. (CI)
 * for the collision (memory) integrals and eq. (2BSE) for the second-Born
 * self-energy, on the k grid of eq. (kj). Every step of the path runs in HIP
 * kernels on the caller's stream; there is no host fallback.
 *
 * Conventions
 *   G^<(t,t') = i<c^dag(t') c(t)>, G^>(t,t') = -i<c(t) c^dag(t')>,
 *   G(t',t) = -[G(t,t')]^dag, rho(t) = -i G^<(t,t).
 *   k grid: k_j = -pi + 2 pi j / n per axis (eq. (kj), 0-based j); flattened k = ix*nky + iy.
 *   Complex numbers are two doubles (re, im), interleaved.
 *
 * Memory ownership
 *   All device memory is allocated by the caller (e.g. as torch tensors) with the
 *   sizes returned by kbe_workspace_query, and must outlive the context. The library
 *   allocates no device memory. Host pointers passed to a call are read before the
 *   call returns.
 *
 * Errors
 *   Every int-returning function returns KBE_OK (0) or a negative KBE_ERR_* code;
 *   kbe_last_error gives a message for the last failing call on a context. Calls
 *   that only enqueue work (kbe_step, kbe_stage_*) report launch errors immediately
 *   and kernel-side faults at the next synchronising call.
 */
#ifndef KBE_H_
#define KBE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  KBE_OK = 0,
  KBE_ERR_INVALID_ARG = -1,  /* null pointer, out-of-range parameter */
  KBE_ERR_SHAPE = -2,        /* unsupported sizes (nb, grid, nt_max) */
  KBE_ERR_HIP = -3,          /* a HIP runtime call failed */
  KBE_ERR_STATE = -4,        /* call out of order (e.g. stepping past nt_max) */
  KBE_ERR_NONFINITE = -5,    /* a NaN/Inf appeared in the propagated state */
  KBE_ERR_NOT_CONVERGED = -6 /* kbe_step: the corrector's stopping rule (corr_tol > 0) ran all n_corr
                                passes with the row still changing by more than corr_tol */
};

/* Interaction presets (eq. (ham) and eq. (2BSE)). */
enum {
  KBE_INT_HUBBARD = 0,   /* spin-degenerate, intra-orbital on-site U: Sigma_ab = U^2 G_ab G_ab G_ba */
  KBE_INT_INTERBAND = 1  /* the paper's spinless two-band model (nb = 2): direct - exchange, with the
                            -U n_c one-body term of eq. (ham) and its Hartree-Fock field (U n_c on v,
                            U n_v on c, -U rho_vc between them). The workspace then holds the
                            real-space lines of the current row, (nt_max + 1) * 8 * N_k complex. */
};

/* Precision of the stored history and of the history sums (the rest of the step is FP64 in
 * every form): KBE_FP64; KBE_FP32, FP32 storage summed on the vector ALU; KBE_FP32_MFMA, FP32
 * storage in the quad layout below, the column sums of eq. (CI) on the FP32 matrix cores with
 * the self-energy row split into FP32 hi + lo parts (compensated products, FP32 accumulation
 * over 32-row tiles, FP64 across tiles) and the row sums on the vector ALU in FP32. */
enum { KBE_FP64 = 0, KBE_FP32 = 1, KBE_FP32_MFMA = 2 };

/* Observable columns of the per-step time series (see kbe_observables). */
enum {
  KBE_OBS_T = 0,      /* time t_m = m dt */
  KBE_OBS_N = 1,      /* particles per site, s/N_k sum_k tr rho */
  KBE_OBS_EKIN = 2,   /* s/N_k sum_k tr[h0(k - A) rho] */
  KBE_OBS_EHF = 3,    /* s/(2 N_k) sum_k tr[Sigma^HF rho] */
  KBE_OBS_ECORR = 4,  /* -(i/2) s/N_k sum_k tr I^<(t,t) (Galitskii-Migdal) */
  KBE_OBS_ETOT = 5,
  KBE_OBS_JX = 6,     /* s/N_k sum_k tr[v_x(k - A) rho] */
  KBE_OBS_JY = 7,
  KBE_OBS_A = 8,      /* pulse amplitude A(t_m) */
  KBE_OBS_NORB = 9,   /* 4 columns: orbital occupations per spin N_k^-1 sum_k rho_aa */
  KBE_OBS_NBAND = 13, /* 4 columns: band occupations per spin in the eigenbasis of h0(k - A), ascending */
  KBE_NOBS = 17
};

/* Workload description (plain data; the caller keeps ownership). */
typedef struct {
  int32_t nkx, nky;     /* k grid; nky = 1 is a 1D chain of 1..1024 points, otherwise a 2D grid with
                           nkx, nky <= 64 and nkx*nky <= 1024 */
  int32_t nb;           /* orbitals per spin, 1..4 (interband preset: 2) */
  int32_t spin_deg;     /* 1 or 2: prefactor s of the observables */
  int32_t interaction;  /* KBE_INT_* */
  int32_t hf;           /* 1: include the first-order (Hartree-Fock) self-energy in h */
  int32_t corr;         /* 1: include the second-Born correlation self-energy */
  int32_t n_corr;       /* corrector passes K per step (>= 0); a step costs K+1 history passes.
                           With corr_tol > 0 the most passes a step may take. */
  int32_t nt_max;       /* largest step index the buffers hold */
  int32_t precision;    /* KBE_FP64, KBE_FP32 or KBE_FP32_MFMA: history stored and summed in FP32 */
  int32_t quad_points;  /* quadrature of eq. (CI): 0 or 1 = the trapezoid rule (the second-order
                           quadrature of Sec. "Computational Kernels"); q = 2..6 = Gregory end corrections on q
                           nodes per end of each interval [0, N]: node j weighs
                           1 + c_j [j < q'] + c_{N-j} [N-j < q'], q' = min(q, N + 1), with the c
                           cancelling the Euler-Maclaurin end terms of the trapezoid sum through
                           polynomial degree q' - 1 (q' for odd q'). The adjoint needs q <= 1. */
  double dt, U, temp, filling; /* time step; interaction; initial temperature; electrons per orbital per spin */
  double corr_tol;      /* 0: every step runs n_corr corrector passes. > 0: the stopping rule of
                           Algorithm "prop" (its max and epsilon): after each pass the largest
                           modulus of the change of row m (every t', k, component and orbital
                           pair, the equal-time block included) is brought to the host, and the
                           passes stop once it is <= corr_tol or n_corr passes have run. This
                           synchronises the stream once per pass; kbe_corrector_log reports the
                           passes taken. The adjoint needs corr_tol = 0. */
} kbe_config;

/* Pulse kinds. */
enum {
  KBE_PULSE_PEIERLS = 0,     /* A(t) = amp sin(omega t) exp(-((t - t0)/width)^2) along pol, entering the
                                Bloch Hamiltonian as k -> k - A(t) pol */
  KBE_PULSE_DIPOLE_KICK = 1  /* eq. (dipole): E(t) = amp delta(t - t0) coupling bands 0 and 1 with d_k = 1
                                (nb = 2; omega, width, pol unused). Across the delta G(t0+, t') =
                                K G(t0-, t'), K = cos(amp) 1 - i sin(amp) X (X: ones between bands 0 and
                                1). The kick acts on the slice at the grid time t_{m0} nearest t0
                                (m0 = floor(t0/dt + 1/2)) when that slice is committed (kbe_step,
                                kbe_stage_commit; at m0 = 0 in kbe_create): its observables are the
                                values just before the kick, its row and density matrix are replaced
                                by the kicked ones (K G for t' < t_m0, K G K^dag on the equal-time
                                block), and its self-energy and collision integrals are evaluated
                                again on the kicked row. No vector potential. */
};
typedef struct {
  double amp, omega, t0, width, pol[2];
  int32_t kind;  /* KBE_PULSE_*; kbe_create returns KBE_ERR_INVALID_ARG for an unknown kind, or for a
                    dipole kick with nb != 2, t0 < 0 or a non-finite amp / t0 */
} kbe_pulse;

typedef struct kbe_ctx kbe_ctx;

/*
 * Device layout:
 *   history : G^{<,>}_{ab}(k; t_j, t') for 0 <= t' <= j <= nt_max, packed lower triangle per
 *             k, strip-major and component-interleaved: the columns t' are grouped in strips
 *             of 64; strip s holds rows j = 64 s .. N-1 (N = nt_max + 1), and each row segment
 *             holds the C = 2 nb^2 components one after the other, 64 elements each:
 *               elem(k, c, j, t') = k C P + C (base(s) + 64 (j - 64 s)) + 64 c + (t' - 64 s),
 *               s = t' / 64,  base(s) = 64 s N - 2048 s (s - 1),  P = base(ceil(N / 64)),
 *             c = s * nb^2 + a * nb + b (s = 0: G^<, s = 1: G^>). In the FP32 form the
 *             components of a row segment are stored in pairs interleaved per column:
 *               elem = k C P + C (base(s) + 64 (j - 64 s)) + 128 (c / 2) + 2 (t' - 64 s) + c % 2.
 *             In the FP32-MFMA form (KBE_FP32_MFMA) strip s holds its rows in quads of 4
 *             (Q(s) = ceil((N - 64 s) / 4) quads, the last one padded); inside a quad the 64
 *             columns form 4 groups g of 16, lane L = 16 (j % 4) + (t' % 16), and components
 *             come in pairs ci = c / 2:
 *               elem = k C P + 256 C (qbase(s) + (j - 64 s) / 4) + 2 (64 (g C / 2 + ci) + L) + c % 2,
 *               qbase(s) = s ceil(N / 4) - 8 s (s - 1),  P = 256 qbase(ceil(N / 64)).
 *             Entries above the
 *             diagonal in a strip's first 64 rows are unused. Elements are complex128 (KBE_FP64)
 *             or complex64 (KBE_FP32). In the FP32 form the history sums read the FP32 history
 *             and compute in FP32 (FP32 accumulation over tiles of 16 rows, FP64 across tiles
 *             and strips); rows m-1 and m, the end-point terms, the update, the density matrix
 *             and the observables stay FP64.
 *   workspace: the per-step rows (self-energy row, collision rows, density matrices,
 *             propagators, partial sums); sub-buffers are located with kbe_buffer.
 *   obs     : (nt_max + 1) x KBE_NOBS doubles, row m written when step m completes.
 */
int kbe_workspace_query(const kbe_config* cfg, size_t* history_bytes, size_t* workspace_bytes,
                        size_t* obs_bytes);

/*
 * Create a context and prepare the initial state on the stream (asynchronously): the
 * uncorrelated Fermi-Dirac density of h0(k - A(0)) at temperature cfg->temp, with the
 * chemical potential found by bisection for cfg->filling, row 0 of the history
 * (G^< = i rho0, G^> = -i(1 - rho0)) and the observables of t_0.
 *   hop   : host, 3 complex nb x nb blocks T0, Tx, Ty (row-major, interleaved re/im);
 *           h0(k) = T0 + sum_d (T_d e^{i k_d} + T_d^dag e^{-i k_d}); Ty is ignored when nky = 1.
 *   pulse : host, may be NULL (no pulse).
 *   d_history, d_workspace, d_obs : device buffers and their sizes in bytes; each size must
 *           be at least what kbe_workspace_query returns for the same cfg, else
 *           KBE_ERR_INVALID_ARG and nothing is launched.
 *   hip_stream : hipStream_t to enqueue on (NULL = default stream).
 */
int kbe_create(const kbe_config* cfg, const double* hop, const kbe_pulse* pulse, void* d_history,
               size_t history_bytes, void* d_workspace, size_t workspace_bytes, void* d_obs, size_t obs_bytes,
               void* hip_stream, kbe_ctx** out);

/* Allocation-free variant of kbe_create, for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid allocation): the same context,
 * except that its workspace is not passed in but lives in a static device array of the library,
 * one array of KBE_NOALLOC_WORKSPACE_MAX bytes per device, held from the library's first use
 * on that device until the process ends. The caller passes the history and the observables as
 * for kbe_create. The call allocates no device memory.
 *   - The device is the one current at the call; hip_stream must belong to it.
 *   - KBE_ERR_SHAPE if the workspace of cfg (kbe_workspace_query) exceeds
 *     KBE_NOALLOC_WORKSPACE_MAX (e.g. the 12x12, nb = 2, nt_max = 400 workload needs 86 MiB and
 *     fits; the 24x24, nt_max = 1000 one needs 1.1 GiB and does not); other argument errors as
 *     for kbe_create. Nothing is launched on an error.
 *   - One such context per device at a time: the array is the context's whole state, so a
 *     second kbe_create_noalloc on the device returns KBE_ERR_STATE until kbe_destroy of the
 *     first (which waits for its work to complete) has returned.
 *   - The array keeps the previous context's contents; creation clears the part it uses (a
 *     fill kernel on hip_stream) before it computes the initial state.
 *   - Every other entry point works on the context as on one from kbe_create; kbe_adjoint_attach
 *     still takes a caller-owned adjoint workspace. */
#define KBE_NOALLOC_WORKSPACE_MAX ((size_t)128 << 20)
int kbe_create_noalloc(const kbe_config* cfg, const double* hop, const kbe_pulse* pulse, void* d_history,
                       size_t history_bytes, void* d_obs, size_t obs_bytes, void* hip_stream, kbe_ctx** out);

/* Advance nsteps time steps (Algorithm "prop" with K = cfg->n_corr fixed corrector passes),
 * asynchronously. KBE_ERR_STATE if the step index would pass nt_max. With corr_tol > 0, a step
 * whose n_corr passes all end with the row changing by more than corr_tol is committed as the
 * algorithm commits it, and the call then returns KBE_ERR_NOT_CONVERGED without taking the
 * remaining steps: kbe_current_step is that step, kbe_corrector_log holds its changes, and a
 * further kbe_step call continues from it. */
int kbe_step(kbe_ctx* ctx, int32_t nsteps);

/* Index of the last completed step (0 after kbe_create). */
int32_t kbe_current_step(const kbe_ctx* ctx);

/* Corrector log (host-side record, no synchronisation): for steps first .. first + count - 1,
 * passes[i] = corrector passes taken (0 for step 0 and for steps not yet run); if changes is
 * not NULL, changes[i * n_corr + p] = the row change after pass p of that step (only recorded
 * with corr_tol > 0; -1 where no pass ran). KBE_ERR_INVALID_ARG outside 0 .. nt_max. */
int kbe_corrector_log(const kbe_ctx* ctx, int32_t first, int32_t count, int32_t* passes, double* changes);

/* Synchronise the stream and copy observable rows first..first+count-1 to host_out
 * (count x KBE_NOBS doubles). Returns KBE_ERR_NONFINITE if the state is not finite. */
int kbe_observables(kbe_ctx* ctx, int32_t first, int32_t count, double* host_out);

void kbe_destroy(kbe_ctx* ctx);
const char* kbe_last_error(const kbe_ctx* ctx);

/* ---------------------------------------------------------------------------------------
 * Stage entry points: one call per step of the path, on the context's buffers, for the
 * time slice t_m. kbe_step is the composition
 *   propagators(m, 0); update(m, PREDICT);
 *   K x { sigma(m); collision(m); propagators(m, 1); update(m, CORRECT) };
 *   sigma(m); collision(m); observables(m); commit(m)
 * (the corrector's collision and update are fused inside kbe_step). The observables come
 * before the commit, which applies the dipole kick on its slice.
 * ------------------------------------------------------------------------------------- */

/* Sub-buffers of the workspace (kbe_buffer). */
enum {
  KBE_BUF_SIGMA = 0,  /* [k][3][nb^2][Tp]: Sigma^<, Sigma^>, Sigma^> - Sigma^< of (t_m, t_j), j <= m */
  KBE_BUF_I_PREV = 1, /* [k][C][Tp]: I^{<,>}(t_{m-1}, t'), t' <= m-1 */
  KBE_BUF_I_CUR = 2,  /* [k][C][Tp]: I^{<,>}(t_m, t'), t' <= m */
  KBE_BUF_RHO_PREV = 3, /* [k][nb^2] */
  KBE_BUF_RHO_CUR = 4,
  KBE_BUF_D_PREV = 5,   /* [k][nb^2]: D = I^<(t,t) + I^<(t,t)^dag */
  KBE_BUF_D_CUR = 6,
  KBE_BUF_PROP = 7,     /* [k][3][nb^2]: V = e^{-i hbar dt}, Vh = e^{-i hbar dt/2}, Phi = (V-1) hbar^{-1} */
  KBE_BUF_COL0 = 8,     /* [k][C][q][Tp]: G(t_j, t_i), i < q (q = max(quad_points, 1)): history columns 0..q-1 */
  KBE_BUF_DIAG = 9,     /* [k][C][q][Tp]: G(t_j, t_{j-i}), i < q: the history diagonal band */
  KBE_BUF_ROWS = 10,    /* [R][k][C][Tp]: FP64 copies of the last R = max(2, q) history rows, slot = row % R */
  KBE_NBUF = 11
};
/* Tp = 8 * ceil((nt_max + 1) / 8). Current device pointer and size of a sub-buffer (the
 * _PREV/_CUR roles swap at every completed step). */
int kbe_buffer(const kbe_ctx* ctx, int32_t which, void** ptr, size_t* bytes);

/* Propagators: hbar = h0(k - A(t_{m-1/2})) + Sigma^HF[rho], rho = rho_{m-1} (mode 0) or
 * (rho_{m-1} + rho_m)/2 (mode 1), and V, Vh, Phi per k into KBE_BUF_PROP. */
int kbe_stage_propagators(kbe_ctx* ctx, int32_t m, int32_t mode);

/* Self-energy: second-Born Sigma^{<,>}(k; t_m, t_j), j = 0..m, from history row m (eq. (2BSE)), by
 * batched k <-> R transforms and pointwise products, into KBE_BUF_SIGMA. */
int kbe_stage_sigma(kbe_ctx* ctx, int32_t m);

/* Self-energy as the paper evaluates it (eq. (2BSE) with eq. (polarizability)/(kernel2) for the
 * direct term, O(n_k^2), and the nested momentum sums of Alg. "contraction2" for the exchange
 * term, O(n_k^3) per time pair): the same output as kbe_stage_sigma, into KBE_BUF_SIGMA, for
 * timing the paper's algorithm. Interband preset on a chain with nkx divisible by 8
 * (KBE_ERR_SHAPE otherwise). At n_k = 1024 the slice of 501 time pairs takes about 0.65 s. */
int kbe_stage_sigma_direct(kbe_ctx* ctx, int32_t m);

/* Collision integrals: I^{<,>}(t_m, t'), t' = 0..m (eq. (CI), Langreth left form,
 * trapezoid weights) from history rows 0..m, KBE_BUF_SIGMA, COL0 and DIAG, into
 * KBE_BUF_I_CUR; D_m into KBE_BUF_D_CUR. */
int kbe_stage_collision(kbe_ctx* ctx, int32_t m);

/* Update: row m of the history and rho_m from row m-1:
 * mode 0 (predictor): G(t_m, t') = V G(t_{m-1}, t') + Phi I(t_{m-1}, t'),
 * mode 1 (corrector): same with (I(t_{m-1}, .) + I(t_m, .))/2 (recomputes I(t_m, .) first);
 * rho_m = V rho_{m-1} V^dag - dt Vh Dbar Vh^dag, and the equal-time block. */
int kbe_stage_update(kbe_ctx* ctx, int32_t m, int32_t mode);

/* Observables of t_m from rho_m and I^<(t_m, t_m) into row m of d_obs. */
int kbe_stage_observables(kbe_ctx* ctx, int32_t m);

/* Make step m the current step and swap the _PREV/_CUR roles as kbe_step does after
 * its evaluation pass and observables; m must be the current step + 1 (KBE_ERR_STATE). If m is the slice of a dipole kick
 * (KBE_PULSE_DIPOLE_KICK), first apply the kick to row m and rho_m, and evaluate row m's
 * self-energy and collision integrals again on the kicked row. */
int kbe_stage_commit(kbe_ctx* ctx, int32_t m);

/* Refresh the FP64 working copies (COL0, DIAG, ROWS for rows m-1 and m) from history rows
 * 0..m (after the caller wrote history rows directly). */
int kbe_rebuild_aux(kbe_ctx* ctx, int32_t m);

/* Per-launch timing of the history-sum kernel with HIP events on the context's stream.
 * kbe_timing(ctx, 1) synchronises the stream, clears earlier records and creates the whole
 * event pool up front (two events per history pass of every step up to nt_max), so that no
 * event is created while work is queued; history-sum launches beyond the pool run untimed.
 * kbe_timing(ctx, 0) synchronises and stops recording. kbe_timing_query synchronises and
 * returns the number of timed launches, their summed duration (ms) and the algorithmic bytes
 * they move (each stored history block read once). */
int kbe_timing(kbe_ctx* ctx, int32_t enable);
int kbe_timing_query(kbe_ctx* ctx, int64_t* launches, double* total_ms, double* algo_bytes);

/* ---------------------------------------------------------------------------------------
 * Adjoint (reverse mode) of the propagation. The paper defines the forward map only
 * (Algorithm "prop" with eqs. (Green), (CI), (2BSE)); the adjoint is the exact discrete
 * transpose of that map as the forward kernels evaluate it, so the gradient it returns is
 * the derivative of the computed observable, not of the continuous equations.
 *
 * Loss: one final-time observable O(t_T), T = kbe_current_step at the first adjoint call:
 *   KBE_OBS_NORB + a  (orbital occupation N_k^-1 sum_k rho_aa(T)), or
 *   KBE_OBS_NBAND + b (band occupation in the eigenbasis of h0(k - A(T))).
 * Parameters theta = (pulse amp, pulse omega, U); the initial state does not depend on them.
 *
 * Requirements: precision KBE_FP64, n_corr = 1 with corr_tol = 0, quad_points <= 1, nb <= 2,
 * the Hubbard preset, the Peierls pulse, nkx <= 64, and T >= 1 (KBE_ERR_SHAPE otherwise). The forward run keeps
 * nothing for the adjoint beyond its own history: every committed time slice is a checkpoint.
 * Reversing step m reads rho_{m-1} back from the history diagonal (G^< = i rho exactly) and
 * recomputes I(t_{m-1}, .) with D_{m-1}, the predictor row and the corrector's collision row
 * from the history (unchanged); it overwrites the context's working buffers, so the context
 * cannot be stepped forward afterwards (KBE_ERR_STATE).
 *
 * kbe_adjoint_query: bytes of the caller-owned adjoint workspace for cfg (an FP64 adjoint
 *   history of the same packed shape as the FP64 history, plus per-step rows).
 * kbe_adjoint_attach: hand the workspace (device, >= the queried size) to the context.
 * kbe_adjoint_step: the first call seeds dO/drho(T) (and dO/dA(T)), and every call reverses
 *   one step (t_m -> t_{m-1}), asynchronously. If grad_out is not NULL the call
 *   synchronises and writes the gradient accumulated so far, (dO/damp, dO/domega, dO/dU),
 *   which is final when *steps_remaining == 0. KBE_ERR_STATE once no step remains or the
 *   observable differs from the first call's.
 * ------------------------------------------------------------------------------------- */
int kbe_adjoint_query(const kbe_config* cfg, size_t* adjoint_bytes);
int kbe_adjoint_attach(kbe_ctx* ctx, void* d_adjoint, size_t bytes);
int kbe_adjoint_step(kbe_ctx* ctx, int32_t observable_id, double* grad_out, int32_t* steps_remaining);

#ifdef __cplusplus
}
#endif
#endif /* KBE_H_ */
