/*
 * gipeps.h - C ABI of the gfx950 library for gauge-canonical-form (GCF) PEPS variational Monte
 * Carlo of Z_N lattice gauge theory, pure or coupled to hard-core bosons, on an open L x L square
 * lattice (arXiv:2503.20566).
 *
 * The hot path, per batch of sampled electric-field configurations:
 *   peps_links_from_powers  seeded plaquette powers -> link labels          (input support)
 *   peps_matter_links       occupations + plaquette powers -> configuration  (input support, matter)
 *   peps_sample_init,       Philox-seeded initial states and Metropolis      (input support,
 *   peps_metropolis         sweeps sampling |Psi|^2                           SM S-2 sampling)
 *   peps_metropolis_strip   the same sweeps with strip ratios and environment reuse
 *   peps_project            Gauss-law check, block selection, gather         (eq. A, eq. gcf, SM S-2)
 *   peps_amplitude          boundary-MPS contraction -> ln|Psi|, sign        (SM S-2 eq. project)
 *   peps_amplitude_noalloc  the same without a workspace (fixed in-library scratch)
 *   peps_amplitude_ragged   the same for several lattices, one launch per boundary row
 *   peps_local_energy       E_loc of the plaquette + electric Hamiltonian     (SM S-1 eq. Es)
 *   peps_eloc_scale         magnitude sum |term| of each E_loc                (SM S-1 eq. Es)
 *   peps_logderiv           O_k = d ln|Psi| / d theta_k                      (SM S-1, O_m)
 *   sr_build                SR force F, mean <O>, and S or S*v                (SM S-1 eq. gradient, SM S-3)
 *   sr_dense_rows           row blocks of the dense S for any parameter count   (SM S-3)
 *   sr_solve                (S + shift I) x = F by conjugate gradients         (SM S-1, SM S-3)
 *   peps_autotune           row-sweep tuning timed on the caller's batch (peps_get/set_tuning)
 *   peps_cx_*, tvmc_rhs,    complex tensors, exact contraction, the tVMC      (SM S-3)
 *   tvmc_step               velocity and the two-stage time step
 *
 * Conventions shared by every call
 *   - Lattice: vertices (x, y), 0 <= x, y < L.  links is uint8 [B][P][L][L] with P = 2 planes (3
 *     with matter): links[b][0][y][x] is the horizontal link (x,y)-(x+1,y), links[b][1][y][x] the
 *     vertical link (x,y)-(x,y+1); slots x = L-1 of plane 0 and y = L-1 of plane 1 are ignored.
 *     Labels are in [0, N).  With matter, links[b][2][y][x] = p(x,y) in {0, 1} is the hard-core
 *     boson occupation of vertex (x,y) (any other value makes the configuration unphysical).
 *   - Gauss law at (x,y): (p + n_l + n_d - n_r - n_u) mod N == Q[y*L+x] (eq. gauss_N; p = 0
 *     without matter).
 *   - Plaquette p = (px, py) (lower-left vertex): P_p raises h(px,py) and v(px+1,py) and lowers
 *     h(px,py+1) and v(px,py) (eq. H_b operator order).
 *   - Parameters theta (float64 [n_params]): sites row-major (y*L+x); in a site, the legs present
 *     in (l, r, d, u) order; blocks = charge tuples of the present legs in lexicographic order that
 *     obey eq. A with p = 0, then (with matter) those that obey it with p = 1; entries of a block
 *     row-major in (l, r, d, u); absent legs have dimension 1.  peps_param_layout reports the
 *     count and per-site offsets.
 *   - Projected tensors proj: float64 [B][L*L][Dk^4]; the selected block of site s occupies the
 *     first Dk^(#present legs) entries of row s (rest zero).  block_id: int32 [B][L*L], the
 *     block's index inside its site, -1 at a vertex that violates the Gauss law.
 *   - The contraction (peps_amplitude) is defined by this algorithm (the paper leaves the
 *     compression open; this is the reading used here): B_0 = row 0 as an MPS; for y = 1..L-2 apply
 *     row y exactly (boundary bond major in each fused bond), sweep reduced QR left to right, sweep
 *     SVD right to left keeping k = min(chi, rows, cols) largest singular values, divide by the
 *     state norm nu_y; close with row L-1 exactly.  ln|Psi| = sum ln nu_y + ln|c|, sign = sign(c).
 *   - Variational compression (var_sweeps = k > 0): after step "SVD sweep" of a row, the truncated
 *     MPS G (bonds kept, right-canonical) is refined by k sweeps, each left to right then right to
 *     left: at site c the tensor C = L_c M_c R_{c+1} (M the exact product of the row with the
 *     previous boundary, L and R the overlaps of G's canonical sites with M) replaces G_c, split by a
 *     reduced QR into the canonical site (left to right Q, right to left Q^T of the QR of C^T) with
 *     the pass's last site keeping C; then nu_y = ||C|| of the final site 0.  Applied to the down
 *     rows of peps_amplitude, the up rows of peps_local_energy and both in peps_metropolis_strip.
 *   - Local energy: E_loc(s) = sum_l e[n_l] + sum_p sum_{t=1}^{N-1} c[t] Psi(P_p^-t s)/Psi(s); the
 *     ratio of plaquette p is taken on the two-row strip (py, py+1) contracted exactly between s's
 *     own down boundary D_{py-1} and up boundary U_{py+2}.  With matter (eq. matter, uniform
 *     m_x = mass, coupling J = hop) E_loc adds mass * sum_x p_x and, for each link whose ends
 *     differ in occupation, hop * Psi(s')/Psi(s) with s' = s after the boson crossed the link (the
 *     link raised when the boson moved towards -x / -y, lowered otherwise); that ratio is taken on
 *     the strip and two-column window holding both ends (a horizontal link of row y: strip
 *     min(y, L-2), its own column; a vertical link (x,y)-(x,y+1): strip y, column min(x, L-2)).
 *
 * Memory and errors
 *   - Every pointer argument except the handle, the problem and host tables is a DEVICE pointer
 *     owned by the caller.  Calls are asynchronous on `stream` (a hipStream_t, NULL = default
 *     stream); outputs are ready when the stream reaches them.
 *   - Graph capture: the first call of a handle on a device uploads its tables (allocation and
 *     copy); after that peps_links_from_powers, peps_project, peps_amplitude, peps_local_energy,
 *     peps_logderiv, sr_build and peps_flags only launch kernels and device-to-device copies on
 *     `stream` (no allocation, synchronisation or memset), so a step may be captured into a HIP
 *     graph and replayed with new inputs in the captured buffers.  sr_solve reads residuals back
 *     to the host each iteration and cannot be captured.
 *   - Each call returns a status (PEPS_OK = 0).  Argument, shape and workspace errors are detected
 *     on the host before anything is launched; a HIP launch failure returns PEPS_ERR_HIP.
 *     Nothing aborts and no exception crosses the ABI.  peps_status_string gives a message.
 *   - Per-sample numerical outcomes are data, not errors: a configuration that violates the Gauss
 *     law has valid = 0, log_abs = -inf, sign = 0, e_loc = NaN and O = 0.
 *   - B = 0 is accepted by every call and does nothing (no output is written, pointers may be
 *     NULL).  sr_build and sr_solve over a batch with no valid sample give F = O_mean = 0 and S = 0
 *     (S v = 0, x = 0).
 *   - Supported shapes: 2 <= L <= 64, 2 <= N <= 8, uniform degeneracy deg[k] = Dk for all k < N
 *     with 1 <= Dk <= 2, 1 <= chi and largest fused bond chi * Dk <= 72 on every entry point.
 *     Fused bonds from 73 to 128 (Dk = 2, chi <= 64: the Z4 32 x 32, D = 8, chi = 64 study; SM
 *     S-4) run on large-bond kernels whose working matrices live in the workspace rather than in
 *     LDS: every real-tensor entry point except peps_amplitude_noalloc, which refuses such a
 *     handle (their row kernel always runs four Jacobi lanes per column pair, whatever
 *     peps_tuning says); such a problem with keep_tape or var_sweeps is refused by peps_create.
 *     Other shapes return PEPS_ERR_UNSUPPORTED.
 */
#ifndef GIPEPS_H
#define GIPEPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PEPS_OK = 0,
  PEPS_ERR_ARG = 1,         /* null pointer, negative size or value out of range */
  PEPS_ERR_UNSUPPORTED = 2, /* valid problem outside the shapes the library supports */
  PEPS_ERR_WORKSPACE = 3,   /* workspace pointer missing or smaller than required */
  PEPS_ERR_HIP = 4,         /* a HIP runtime call or kernel launch failed */
  PEPS_ERR_STATE = 5        /* a call that needs an earlier call's results in ws came first */
};

enum { PEPS_F64 = 0, PEPS_F32_MIXED = 1, PEPS_C128_EXACT = 2, PEPS_C64_EXACT = 3 };

/* Workspace parts, OR-ed into `what` of peps_workspace_bytes. */
enum { PEPS_WS_AMPLITUDE = 1, PEPS_WS_ENERGY = 2, PEPS_WS_LOGDERIV = 4, PEPS_WS_SAMPLE = 8,
       PEPS_WS_TVMC = 16 };

/* Sample weights of the tVMC averages: plain means over the valid samples (Metropolis samples), or
 * |Psi|^2 normalised over them (an enumeration of every configuration of a small lattice). */
enum { TVMC_WEIGHT_UNIFORM = 0, TVMC_WEIGHT_PSI2 = 1 };

/* sr_build modes */
enum { SR_MATVEC = 0, SR_DENSE = 1 };

/* Per-sample flag bits (peps_flags). */
enum { PEPS_FLAG_SVD_NOCONV = 1 };

typedef struct {
  int32_t L, N;         /* L x L vertices, open boundary; gauge group Z_N                       */
  int32_t deg[8];       /* D_k, degeneracy of charge sector k (eq. A; D = sum_k D_k)            */
  int32_t chi;          /* boundary-MPS cutoff (VMC section)                                     */
  const int8_t* Q;      /* HOST [L*L] background charges Q_x (eq. gauss_N), NULL = all zero      */
  double plaq_coef[8];  /* c[t], t = 1..N-1: H_B = sum_p sum_t c[t] P_p^t; c[t] == c[N-t]          */
  double elec[8];       /* e[n], n = 0..N-1: H_E = sum_l e[n_l] (eq. electric is one choice)     */
  int32_t dtype;        /* PEPS_F64, or PEPS_F32_MIXED: the product of a boundary row with the
                         * next PEPS row in FP32 (inputs prescaled by a power of two), every
                         * factorisation, the strips and the adjoint in FP64; or
                         * PEPS_C128_EXACT: complex tensors, exact contraction, the peps_cx_*
                         * and tvmc_* calls only (see there); PEPS_C64_EXACT: the same with the
                         * contractions in complex64                                          */
  int32_t ckpt_every;   /* peps_logderiv: keep every k-th boundary row, recompute the rest (0 = all) */
  int32_t keep_tape;    /* 1: peps_amplitude stores every row's factorisations in ws and
                         * peps_logderiv reverses them without recomputing the rows (needs
                         * ckpt_every <= 1; PEPS_WS_AMPLITUDE then grows by about
                         * (L-2) * L * 5 * (chi*Dk)^2 doubles per sample); 0: recompute      */
  int32_t max_sweeps;   /* Jacobi sweep limit per truncated SVD (0 = 40); a sample whose SVD
                         * stops at the limit unconverged gets PEPS_FLAG_SVD_NOCONV (peps_flags) */
  int32_t matter;       /* 1: hard-core bosons on the vertices (eq. matter; configurations carry
                         * the occupation plane, the layout the p = 1 blocks); 0: pure gauge  */
  double hop;           /* J of eq. matter, coefficient of c^dag_x U_(x,a) c_(x+e_a) + h.c.     */
  double mass;          /* m_x of eq. matter (uniform); hop = mass = 0 unless matter = 1         */
  int32_t var_sweeps;   /* variational compression (SM S-2 "SVD or variational compression"): 0
                         * = the SVD truncation alone; k > 0 (<= 100) = each truncated boundary
                         * row refined by k sweeps of single-site updates maximising its overlap
                         * with the exact row product (the fitting algorithm; see below).  Not
                         * with keep_tape, complex tensors, peps_logderiv or
                         * peps_amplitude_noalloc (PEPS_ERR_UNSUPPORTED)                      */
} peps_problem;

typedef struct peps_handle peps_handle;

/* Validate the problem and build the host and device tables (layout offsets, bond dimensions)
 * on the current HIP device.  The handle owns only these tables; free with peps_destroy. */
int peps_create(const peps_problem* prob, peps_handle** out);
int peps_destroy(peps_handle* h);
const char* peps_status_string(int status);

/* n_params (HOST int64*) and, if site_offset (HOST int64 [L*L+1]) is not NULL, the per-site
 * offsets of the layout described above. */
int peps_param_layout(const peps_handle* h, int64_t* n_params, int64_t* site_offset);

/* Bytes of device workspace a batch of B needs for the parts in `what` (PEPS_WS_*).  One buffer
 * sized for AMPLITUDE|ENERGY|LOGDERIV serves every call; peps_local_energy and peps_logderiv
 * read the boundary rows that peps_amplitude left in it, so pass the same buffer to all three. */
int peps_workspace_bytes(const peps_handle* h, int32_t B, uint32_t what, size_t* bytes);

/* Input support (not part of the timed path): links = prod_p P_p^{k_p} |0>, i.e.
 * h(x,y) = k(x,y) - k(x,y-1), v(x,y) = k(x-1,y) - k(x,y) mod N with out-of-range k = 0.
 * powers: uint8 [B][L-1][L-1] indexed [py][px]; links: uint8 [B][P][L][L] (with matter the
 * occupation plane is written empty). */
int peps_links_from_powers(peps_handle* h, const uint8_t* powers, int32_t B, uint8_t* links,
                           void* stream);

/* Input support for matter problems (not part of the timed path): a configuration with the given
 * occupations that obeys the Gauss law (eq. gauss_N), times prod_p P_p^{k_p}.  The flux carries
 * each vertex's charge Q_x - p_x along its row to column 0 and down column 0:
 * h(x,y) = sum_{x'>x} (Q - p)(x',y), v(0,y) = sum_{y'>y, all x'} (Q - p), other vertical links 0,
 * then the plaquette powers' closed form above (mod N).  Vertex (0,0) obeys the Gauss law only if
 * sum_x p_x = sum_x Q_x (mod N); otherwise that sample projects as unphysical (data, not an error).
 * powers: uint8 [B][L-1][L-1]; occupations: uint8 [B][L][L]; links: uint8 [B][3][L][L].
 * PEPS_ERR_ARG on a handle without matter. */
int peps_matter_links(peps_handle* h, const uint8_t* powers, const uint8_t* occupations, int32_t B,
                      uint8_t* links, void* stream);

/* SM S-2, configuration sampling (input support that generates Metropolis-sampled workloads; not
 * part of the timed path).  The paper fixes no generator; this library uses the counter-based
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) with key = (seed, stream_id) and counter =
 * (chain b, sweep w, plaquette p, purpose); a draw is the first 64-bit output word x and
 * u = (x >> 11) * 2^-53.  Plaquettes p = py (L-1) + px are visited in that order.
 * With matter, link moves move the bosons (SM S-2; eq. matter's hopping): the move of link (d,x,y)
 * proposes s' = s with the boson moved across it when exactly one end is occupied (the link raised
 * when the boson moves towards -x / -y, lowered otherwise), and is skipped, drawing nothing, when
 * both ends hold the same occupation.  Its uniform is the draw of counter (b, w, (L-1)^2 + index, 2)
 * with index y (L-1) + x for a horizontal and L (L-1) + y L + x for a vertical link.  The links of
 * strip py (vertical links of row py, horizontal links of row py and, for py = L-2, of row L-1) are
 * visited right after plaquette row py, by window column px = 0 .. L-2: vertical (px, py),
 * horizontal (px, py), horizontal (px, L-1) when py = L-2, and vertical (L-1, py) when px = L-2.
 *
 * peps_sample_init: chain b starts at prod_p P_p^{k_p} |0> with k_p = x mod N, x the draw of
 * counter (b, 0, p, 0).  powers: uint8 [B][L-1][L-1] and links: uint8 [B][2][L][L] (layouts of
 * peps_links_from_powers), both written.  These states lie in the Q = 0 sector; with background
 * charges the chains start from caller-supplied links of the charged sector instead (plaquette
 * moves keep every vertex's Gauss residual, so peps_metropolis stays in that sector).  A matter
 * problem returns PEPS_ERR_UNSUPPORTED: its chains start from peps_matter_links. */
int peps_sample_init(peps_handle* h, uint64_t seed, uint64_t stream_id, int32_t B, uint8_t* powers,
                     uint8_t* links, void* stream);

/* Metropolis sweeps w = first_sweep .. first_sweep + n_sweeps - 1 of every chain: at each plaquette
 * the proposal s' = P_p^t s with t = 1 + x mod (N-1) (purpose 1) is accepted iff
 * u < exp(2 (ln|Psi(s')| - ln|Psi(s)|)) (purpose 2, float64), with ln|Psi| from peps_project and
 * peps_amplitude of this handle (one amplitude per proposal and chain; for a complex handle,
 * PEPS_C128_EXACT or PEPS_C64_EXACT, from peps_cx_project and peps_cx_amplitude, theta complex, proj sized as peps_cx_project
 * writes it, ws for PEPS_WS_AMPLITUDE|PEPS_WS_SAMPLE of that handle); with matter, each
 * plaquette row is followed by its strip's link moves under the same rule.  links: uint8
 * [B][P][L][L], the chains' states, read and overwritten with the final states; log_abs: float64 [B], written
 * with ln|Psi| of the final states; accepted: int32 [B] or NULL, the accepted proposals of each
 * chain are added to it.  theta as for peps_project; proj, block_id, valid: caller scratch of the
 * sizes peps_project writes.  ws: sized for PEPS_WS_AMPLITUDE|PEPS_WS_SAMPLE.  The boundary rows
 * left in ws belong to a proposal: call peps_amplitude on the final links before
 * peps_local_energy or peps_logderiv (they return PEPS_ERR_STATE until then). */
int peps_metropolis(peps_handle* h, const double* theta, uint64_t seed, uint64_t stream_id,
                    int32_t first_sweep, int32_t n_sweeps, int32_t B, uint8_t* links, double* log_abs,
                    int32_t* accepted, double* proj, int32_t* block_id, uint8_t* valid, void* ws,
                    size_t ws_bytes, void* stream);

/* SM S-2 configuration sampling with strip ratios (the finite-PEPS form of the sweep: each ratio is
 * taken on the two-row strip of its plaquette with the environments of the local energy, and the
 * environments are reused along the sweep).  Same generator, counters and rule as peps_metropolis,
 * with |Psi(s') / Psi(s)| replaced by |Psi_py(s') / Psi_py(s)|, Psi_py the strip amplitude
 * <U_{py+2}| row py+1, row py |D_{py-1}> of plaquette (px, py), D and U the canonical boundaries of
 * the current configuration.  Plaquette rows are visited upwards on odd sweep indices w and
 * downwards on even ones (px ascending within a row), so each pass builds, behind it, the
 * boundaries the next pass needs: per strip the right environments, then per plaquette the
 * proposal's ratio from the left environment, the decision and the left environment after it;
 * after each strip one boundary row (D_py going up, U_{py+1} going down).  With matter, the
 * strip's link moves follow its plaquettes in a second pass over the strip (right environments of
 * the updated strip, then per window column its link moves against the left environment, which
 * advances after the column's last decision).  A call first builds the
 * boundaries its first sweep needs.  When chi is exact the strip ratio equals the amplitude ratio.
 * Cost per sweep: one boundary sweep and L-1 strips, against one boundary sweep per proposal for
 * peps_metropolis.
 * Arguments as peps_metropolis; ws: sized for PEPS_WS_AMPLITUDE|PEPS_WS_ENERGY.  On return
 * log_abs holds ln|Psi| of the final states and ws the state peps_amplitude leaves for them, so
 * peps_local_energy and peps_logderiv may follow directly (peps_flags then reports the SVDs of that
 * final amplitude).
 * Complex handles (PEPS_C128_EXACT, PEPS_C64_EXACT): every sweep visits the plaquette rows upwards,
 * the order of peps_metropolis, with the exact ratio of the complex local energy (the row pair of
 * the plaquette between the row state below it and the one above it, the lower rows re-contracted
 * as the chain moves); the decisions are those of peps_metropolis on the same chains up to the
 * rounding of the ratio.  Per sweep: one peps_cx_amplitude and one pass of the local energy's
 * cost.  theta, proj as for peps_cx_project; ws: sized for PEPS_WS_AMPLITUDE|PEPS_WS_SAMPLE; on
 * return ws holds the row states of the final chains (peps_cx_local_energy, peps_cx_logderiv may
 * follow). */
int peps_metropolis_strip(peps_handle* h, const double* theta, uint64_t seed, uint64_t stream_id,
                          int32_t first_sweep, int32_t n_sweeps, int32_t B, uint8_t* links,
                          double* log_abs, int32_t* accepted, double* proj, int32_t* block_id,
                          uint8_t* valid, void* ws, size_t ws_bytes, void* stream);

/* eq. A / eq. gcf / SM S-2: check the Gauss law at every vertex, select each site's block from its
 * link labels and gather it.  theta: float64 [n_params]; outputs proj, block_id, valid as above. */
int peps_project(peps_handle* h, const double* theta, const uint8_t* links, int32_t B,
                 double* proj, int32_t* block_id, uint8_t* valid, void* stream);

/* SM S-2 eq. project with the boundary algorithm above.  log_abs, sign: float64 [B].  Leaves the
 * boundary rows D_0..D_{L-2} and their ln nu_y in ws (needs PEPS_WS_AMPLITUDE). */
int peps_amplitude(peps_handle* h, const double* proj, const uint8_t* valid, int32_t B,
                   double* log_abs, double* sign, void* ws, size_t ws_bytes, void* stream);

/* Ragged batch (VMC section and SM S-4: the lattices of one study, e.g. 8 x 8, 12 x 12 and 24 x 24,
 * sampled together): for every group i < n the same as peps_amplitude(h[i], proj[i], valid[i],
 * B[i], log_abs[i], sign[i], ws[i], ws_bytes[i], stream), but boundary row y of every lattice that
 * has it (1 <= y <= L_i - 2) is computed in one launch, the workgroups of all groups together.
 * 1 <= n <= 8; all handles real, of one dtype and D_k = 2, without keep_tape or var_sweeps
 * (PEPS_ERR_UNSUPPORTED otherwise), either all or none with fused bonds above 72; each ws[i]
 * sized for h[i] with PEPS_WS_AMPLITUDE (checked, PEPS_ERR_WORKSPACE).  The row kernel is the one
 * selected by the largest fused bond of the groups, with the Jacobi lanes, waves and
 * preconditioning of h[0]'s tuning: a group whose own kernel differs gets ln|Psi| equal to its
 * peps_amplitude result up to rounding (identical bits where the kernels agree).  Afterwards each
 * ws[i] is in the state peps_amplitude leaves (peps_local_energy / peps_logderiv may follow on it).
 * Groups with B[i] = 0 are skipped.  A handle may be listed more than once, each time with its own
 * workspace (groups that share a workspace race). */
int peps_amplitude_ragged(int32_t n, peps_handle* const* h, const double* const* proj,
                          const uint8_t* const* valid, const int32_t* B, double* const* log_abs,
                          double* const* sign, void* const* ws, const size_t* ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): peps_amplitude without a workspace.  Same kernels, same
 * results (log_abs, sign bit-identical to peps_amplitude's on the same inputs); the scratch
 * (two boundary rows used alternately, ln nu_y, the Q factors of the row being swept, flag
 * words) is a fixed 128 MiB array inside the library, one per GPU, held until the process ends.
 * A batch needs about B * 8 * (2 * L * chi^2 * Dk + L * Dk * M^2 + L) bytes (M = 72 when
 * chi * Dk > 32, else 32): B up to 67 at L = 16, chi = 36, Dk = 2; a larger batch returns
 * PEPS_ERR_WORKSPACE before anything runs.  Fused bonds above 72 are refused
 * (PEPS_ERR_UNSUPPORTED).  Nothing is allocated, freed or
 * set with hipMemset: the call only launches kernels on `stream`.  The handle's tables must be on
 * the current device (peps_create puts them there when a GPU is present; PEPS_ERR_STATE if not,
 * PEPS_ERR_ARG for another device).  Nothing is left for peps_local_energy / peps_logderiv.
 * Every call on one GPU uses the same array: calls that overlap in time on one GPU (other
 * streams, other threads, other handles) race and must be serialised by the caller. */
int peps_amplitude_noalloc(peps_handle* h, const double* proj, const uint8_t* valid, int32_t B,
                           double* log_abs, double* sign, void* stream);

/* SM S-1 eq. Es.  theta, links and proj of the same batch (theta supplies the blocks that the
 * plaquette moves select); e_loc: float64 [B].  Needs the ws of the preceding peps_amplitude on the
 * same batch (sized for PEPS_WS_AMPLITUDE|PEPS_WS_ENERGY); returns PEPS_ERR_STATE when the last
 * peps_amplitude on this handle used another ws or batch size.  Runs the mirrored (up) boundary
 * sweep, then one strip kernel per row pair. */
int peps_local_energy(peps_handle* h, const double* theta, const uint8_t* links,
                      const double* proj, const uint8_t* valid, int32_t B, double* e_loc,
                      void* ws, size_t ws_bytes, void* stream);

/* SM S-1: O_k(s) = d ln|Psi(s)| / d theta_k of the amplitude defined above: the exact derivative of
 * every step (row application, QR, truncated SVD with its kept-discarded coupling terms,
 * normalisation, close), by a hand-written reverse sweep that recomputes each row's factorisations
 * from the stored boundary rows.  With ckpt_every = k > 1 only rows y = 0 mod k are read from ws and
 * the rows between are recomputed; with keep_tape = 1 nothing is recomputed: the factorisations
 * that peps_amplitude stored in ws are reversed directly (same bits as the recompute).  O: float64 [B][L*L][Dk^4] in the projected layout (derivative
 * w.r.t. the selected block entries; every other parameter has O_k = 0; padding and invalid samples
 * are 0), required.  vjp: float64 [n_params] = sum_b w[b] O_b scattered through block_id (w NULL =
 * all ones; valid samples only), or NULL.  Needs the ws of the preceding peps_amplitude on the same
 * batch (sized for PEPS_WS_AMPLITUDE|PEPS_WS_LOGDERIV), else PEPS_ERR_STATE.  Requires nonzero
 * kept singular values and invertible R factors at every step (true for generic tensors). */
int peps_logderiv(peps_handle* h, const double* proj, const int32_t* block_id,
                  const uint8_t* valid, int32_t B, const double* w, double* O, double* vjp,
                  void* ws, size_t ws_bytes, void* stream);

/* SM S-1 eq. gradient (read as the covariance <O E> - <O><E>, the printed equation repeating one
 * term) and SM S-3 S_mn = <O_m O_n> - <O_m><O_n>, plain means over the valid samples.
 * O, block_id: as produced by peps_logderiv.  F, O_mean: float64 [n_params].
 * mode SR_MATVEC: v float64 [n_params] input, S_or_Sv float64 [n_params] = S v (what a conjugate-
 *                 gradient solve needs; S is never formed).
 * mode SR_DENSE:  v unused, S_or_Sv float64 [n_params][n_params] row-major = S; only for
 *                 n_params <= 8192 (PEPS_ERR_UNSUPPORTED otherwise).
 * ws: the workspace of peps_workspace_bytes(..., PEPS_WS_LOGDERIV) (uses B + 8 doubles of it).
 * Reductions run over samples in index order: results are bitwise reproducible. */
int sr_build(peps_handle* h, const double* O, const int32_t* block_id, const uint8_t* valid,
             const double* e_loc, int32_t B, int32_t mode, const double* v, double* F,
             double* O_mean, double* S_or_Sv, void* ws, size_t ws_bytes, void* stream);

/* SM S-3: rows [row0, row0 + nrows) of the dense S_mn = <O_m O_n> - <O_m><O_n> (plain means over
 * the valid samples), for any parameter count: S has n_params^2 entries (63 GB in float64 at
 * 88,752 parameters), so a dense use of it streams it by row blocks.  O, block_id, valid: as for
 * sr_build; O_mean: float64 [n_params], sr_build's mean for the same batch; S_rows: float64
 * [nrows][n_params] row-major, written.  0 <= row0, 0 <= nrows, row0 + nrows <= n_params.  One
 * workgroup per row adds the samples in index order, each through its selected blocks only: the
 * rows are bitwise those of sr_build's SR_DENSE mode.  No workspace. */
int sr_dense_rows(peps_handle* h, const double* O, const int32_t* block_id, const uint8_t* valid,
                  int32_t B, const double* O_mean, int64_t row0, int64_t nrows, double* S_rows,
                  void* stream);

/* SR parameter update (SM S-1 / SM S-3): solves (S + shift I) x = F by conjugate gradients from
 * x = 0 with the S v products of sr_build's SR_MATVEC mode (S is never formed), stopping when
 * ||F - (S + shift I) x|| <= rtol ||F|| or after max_iter iterations (<= 10000), or at a breakdown
 * p.(S + shift I) p <= 0 (shift >= 0; S is positive semidefinite).  x, F, O_mean: float64
 * [n_params] outputs.  iterations, rel_residual: HOST pointers (or NULL) receiving the iteration count
 * and the final ||r|| / ||F|| (0 when F = 0).  ws: sized for PEPS_WS_LOGDERIV.  Reads one residual
 * per iteration back to the host, so the call synchronises the stream.  Reductions run in a fixed
 * order: results are bitwise reproducible. */
int sr_solve(peps_handle* h, const double* O, const int32_t* block_id, const uint8_t* valid,
             const double* e_loc, int32_t B, double shift, int32_t max_iter, double rtol, double* x,
             double* F, double* O_mean, int32_t* iterations, double* rel_residual, void* ws,
             size_t ws_bytes, void* stream);

/* Per-sample numerical outcomes of the boundary sweeps since the last peps_amplitude on ws (which
 * clears them; the sweeps of peps_local_energy and peps_logderiv on the same ws add theirs):
 * flags uint32 [B], bit PEPS_FLAG_SVD_NOCONV set when a truncated SVD of that sample stopped at
 * the Jacobi sweep limit before converging (its result is then a partial diagonalisation).  An
 * outcome, not an error: the call succeeds.  Copies B words from ws on the stream. */
int peps_flags(peps_handle* h, int32_t B, const void* ws, size_t ws_bytes, uint32_t* flags,
               void* stream);

/* SM S-1 eq. Es, the size of E_loc's terms: scale[b] = sum_l |e[n_l]| + sum_p sum_t |c[t] r_{p,t}|,
 * r_{p,t} the strip ratios that the last peps_local_energy on ws summed (same batch, same rounding).
 * |E_loc| <= scale, and scale is what rounding errors in E_loc are proportional to: an error
 * measured against it cannot shrink when the terms cancel.  float64 [B], NaN for invalid samples.
 * Returns PEPS_ERR_STATE unless the last peps_local_energy on this handle used ws and B and no
 * peps_amplitude ran since.  Copies B doubles from ws on the stream. */
int peps_eloc_scale(peps_handle* h, int32_t B, const void* ws, size_t ws_bytes, double* scale,
                    void* stream);

/* Tuning of the boundary row sweep (the kernel that dominates every call).  None of these choices
 * changes the result beyond rounding: the truncated boundary depends only on the state, and every
 * choice is parity-tested against the oracle.
 *   jacobi_lanes  lanes per column pair in the one-sided Jacobi SVD: 4 or 8
 *   down_precond  large SVDs of the down sweeps (peps_amplitude; reversed by peps_logderiv):
 *                 PEPS_PRECOND_NONE or PEPS_PRECOND_SORTED_QR (columns sorted by norm, QR, Jacobi on
 *                 R^T: the left vectors stay accumulated, as the reverse sweep needs)
 *   up_precond    large SVDs of the up sweeps (peps_local_energy, peps_metropolis_strip):
 *                 PEPS_PRECOND_NONE, PEPS_PRECOND_QR_T (QR of Theta^T, Jacobi on R^T) or
 *                 PEPS_PRECOND_SORTED_QR
 *   precond_min   a cut is preconditioned when Theta is wide or square and its smaller dimension is
 *                 at least this (2 .. 1024)
 *   small_waves   waves per SIMD the kernels for chi * Dk <= 32 are compiled for: 2 (up to 256
 *                 registers, one workgroup per CU) or 4 (128 registers and spills, two per CU)
 * peps_create sets 8, SORTED_QR, QR_T, 16, 2 (the fastest at Z3 16 x 16, chi = 36). */
enum { PEPS_PRECOND_NONE = 0, PEPS_PRECOND_QR_T = 1, PEPS_PRECOND_SORTED_QR = 2 };
typedef struct {
  int32_t jacobi_lanes, down_precond, up_precond, precond_min, small_waves;
} peps_tuning;
/* One timed candidate of peps_autotune: a down (up = 0) or up (up = 1) sweep with the given lanes,
 * preconditioning mode, threshold and waves, ms its duration (HIP events on the stream). */
typedef struct {
  int32_t jacobi_lanes, precond, precond_min, small_waves, up;
  double ms;
} peps_tune_result;

int peps_get_tuning(const peps_handle* h, peps_tuning* t);
/* PEPS_ERR_ARG for a value outside the ranges above.  Changing the tuning invalidates the state a
 * workspace holds (call peps_amplitude again before peps_local_energy / peps_logderiv). */
int peps_set_tuning(peps_handle* h, const peps_tuning* t);
/* Autotuner: times, on the caller's batch (proj, valid of peps_project, B > 0), one down sweep and
 * one up sweep for each candidate -- jacobi_lanes in {8, 4} x precond_min in {16, 32} (x
 * small_waves in {2, 4} when the chi * Dk <= 32 kernels run), each with every down mode and every
 * up mode -- and keeps, over those combinations, the fastest down mode plus the fastest up mode
 * with the smallest sum; that tuning is set on the handle and returned in *best.  results (HOST,
 * capacity entries, or NULL with capacity 0) receives the timings in the order run, *count (HOST,
 * or NULL) their number (20, or 40 with the waves).  ws: sized for PEPS_WS_AMPLITUDE |
 * PEPS_WS_ENERGY; its contents are overwritten and the workspace state is invalidated as by
 * peps_set_tuning.  Synchronises the stream after every candidate; allocates two HIP events. */
int peps_autotune(peps_handle* h, const double* proj, const uint8_t* valid, int32_t B, void* ws,
                  size_t ws_bytes, peps_tuning* best, peps_tune_result* results, int32_t capacity,
                  int32_t* count, void* stream);

/* ---------------------------------------------------------------------------------------------
 * Complex tensors and real-time evolution (SM S-3: eq. tVMC, S_mn, eq. secondorder), for handles
 * created with dtype = PEPS_C128_EXACT or PEPS_C64_EXACT (the real-path calls above return PEPS_ERR_ARG for them,
 * except the input support and peps_metropolis, which samples |Psi|^2 of the complex amplitude;
 * these calls return PEPS_ERR_ARG for real handles).  Supported: pure gauge (matter = 0, background charges allowed),
 * uniform Dk <= 3, Dk^(L+1) <= 177147 (L <= 16 at Dk = 2, L <= 10 at Dk = 3), keep_tape = 0; chi
 * is not used.  Up to Dk^(L+1) = 2187 a sample's two working states stay in LDS; above, they take a
 * slot of the workspace (2 Dk^(L+1) complex per sample).  Complex numbers are interleaved (re, im) float64 pairs: theta is float64
 * [n_params][2] in the parameter layout above.  PEPS_C64_EXACT runs the contractions (row states,
 * site absorptions, environments) in complex64, with the row states' power-of-two exponents, the
 * overlaps and ratios, ln|Psi|, and every input and output in float64 as above; the workspace's
 * row states then take half the bytes.
 *
 * Reading: a truncated SVD is not a holomorphic function of the tensors, so O_m = d ln Psi /
 * d alpha_m is taken on the exact amplitude: the network is contracted row by row in the full space
 * of a row cut's vertical bonds (Dk^L states; each row applied one site at a time, every row state
 * rescaled by an exact power of two), where Psi is multilinear and d Psi / dT_x is the network with
 * site x open.  E_loc uses exact amplitude ratios (eq. Es).
 *
 * peps_cx_project: as peps_project with complex blocks; proj float64 [B][L*L][Dk^4][2] (the block's
 * entries first, in its own shape), block_id, valid as peps_project.
 * peps_cx_amplitude: ln|Psi| (float64 [B]) and the phase Psi/|Psi| (float64 [B][2]); leaves the row
 * states in ws (needs PEPS_WS_AMPLITUDE).
 * peps_cx_local_energy: E_loc float64 [B][2] (NaN for invalid samples); needs the states that
 * peps_cx_amplitude left in ws for this batch (PEPS_ERR_STATE otherwise).
 * peps_cx_logderiv: O float64 [B][L*L][Dk^4][2] in proj's layout (zero beyond each block and for
 * invalid samples); same state requirement. */
int peps_cx_project(peps_handle* h, const double* theta, const uint8_t* links, int32_t B, double* proj,
                    int32_t* block_id, uint8_t* valid, void* stream);
int peps_cx_amplitude(peps_handle* h, const double* proj, const uint8_t* valid, int32_t B, double* log_abs,
                      double* phase, void* ws, size_t ws_bytes, void* stream);
int peps_cx_local_energy(peps_handle* h, const double* theta, const uint8_t* links, const double* proj,
                         const uint8_t* valid, int32_t B, double* e_loc, void* ws, size_t ws_bytes,
                         void* stream);
int peps_cx_logderiv(peps_handle* h, const double* proj, const uint8_t* valid, int32_t B, double* O, void* ws,
                     size_t ws_bytes, void* stream);

/* eq. tVMC: the parameter velocity alphadot solving i (S + shift I) alphadot = g, with sample
 * weights w_b (TVMC_WEIGHT_*, from log_abs and valid), <X> = sum_b w_b X_b,
 * S_mn = <O*_m O_n> - <O*_m><O_n> (SM S-3) applied as S v without forming S, and
 * g_m = <O*_m E_loc> - <O*_m><E_loc> (the covariance reading of eq. gradient).  The Hermitian
 * system (S + shift I) y = g is solved by conjugate gradients from y = 0 until |r| <= rtol |g| or
 * max_iter iterations (<= 10000; the residual norms are read back each iteration, so the call
 * synchronises the stream), and alphadot = -i y.  Inputs as peps_cx_logderiv / peps_cx_local_energy /
 * peps_cx_amplitude wrote them; xdot: float64 [n_params][2]; energy (HOST float64 [2], or NULL):
 * <E_loc>; iterations, rel_residual (HOST, or NULL).  ws: sized for PEPS_WS_TVMC.  shift >= 0. */
int tvmc_rhs(peps_handle* h, const double* O, const int32_t* block_id, const uint8_t* valid, const double* e_loc,
             const double* log_abs, int32_t B, int32_t weights, double shift, int32_t max_iter, double rtol,
             double* xdot, double* energy, int32_t* iterations, double* rel_residual, void* ws, size_t ws_bytes,
             void* stream);

/* One time step of eq. secondorder on the configurations in links (held fixed during the step):
 * order 2: alpha_1 = alpha + c_1 dt alphadot(alpha), alpha <- alpha_1 + c_2 dt alphadot(alpha_1), with
 * c_{1,2} = (1 +- i)/2; order 1: alpha <- alpha + dt alphadot(alpha).  Reading: each stage adds
 * c dt alphadot, alphadot from tvmc_rhs, which is the direction of i d|psi>/dt = H|psi> for the
 * conventions above (the printed update subtracts it).  theta (float64 [n_params][2]) is updated in
 * place; energy (HOST float64 [2], or NULL): <H> = <E_loc> at the start of the step; iterations
 * (HOST int32 [2], or NULL): CG iterations of each stage.  ws: sized for PEPS_WS_TVMC; every
 * intermediate lives there. */
int tvmc_step(peps_handle* h, double* theta, const uint8_t* links, int32_t B, int32_t weights, int32_t order,
              double dt, double shift, int32_t max_iter, double rtol, double* energy, int32_t* iterations,
              void* ws, size_t ws_bytes, void* stream);

/* Per-kernel timing (measurement support).  While enabled, every launch of a hot kernel is
 * bracketed by two HIP events recorded on the launch's own stream.  peps_profile_read waits for
 * the recorded events of one kernel family, returns the number of launches and their summed
 * duration in milliseconds, and forgets them.  Families: PEPS_K_* below. */
enum { PEPS_K_PROJECT = 0, PEPS_K_ROW_SWEEP = 1, PEPS_K_CLOSE = 2, PEPS_K_STRIP = 3,
       PEPS_K_ADJOINT = 4, PEPS_K_SR = 5, PEPS_K_COUNT = 6 };
int peps_profile_enable(peps_handle* h, int32_t on);
int peps_profile_read(peps_handle* h, int32_t family, int64_t* launches, double* total_ms);

/* Phase clocks of the boundary-row kernel (measurement support; the phases of the row step of
 * SM S-2 eq. project and the VMC section's truncation).  counters: DEVICE uint64 [PEPS_PH_COUNT],
 * caller-owned and zeroed by the caller, or NULL to switch the clocks off (the default).  While
 * set, every row-sweep launch of the handle (amplitude, local energy, samplers, ragged batch) adds
 * to counters[p], per workgroup, the shader-clock cycles its first thread spends in phase p:
 * PEPS_PH_X forming X_c = R_{c-1} B_c T_c, PEPS_PH_QR the left-to-right Householder QR (and its
 * tape), PEPS_PH_THETA forming Theta_c = Q_c G_{c+1}, PEPS_PH_PRECOND the QR that preconditions a
 * large SVD (with its column sort), PEPS_PH_JACOBI the one-sided Jacobi sweeps, PEPS_PH_REST the
 * products with the Jacobi's rotations, the truncated outputs, the tape and the last site.  The
 * kernels do the same arithmetic either way.  PEPS_ERR_ARG for a NULL handle. */
enum { PEPS_PH_X = 0, PEPS_PH_QR = 1, PEPS_PH_THETA = 2, PEPS_PH_PRECOND = 3, PEPS_PH_JACOBI = 4,
       PEPS_PH_REST = 5, PEPS_PH_COUNT = 6 };
int peps_profile_phases(peps_handle* h, uint64_t* counters);

#ifdef __cplusplus
}
#endif

#endif /* GIPEPS_H */
