/*
 * laim.h -- C ABI of the MI355X local autonomous inference machine decoder.
 *
 * The library decodes quantum CSS codes with the local machine of
 * "Local autonomous inference machines for quantum LDPC codes": many
 * Monte-Carlo shots run belief propagation (BP) on the Tanner graph of the
 * X-check matrix H (Preliminaries; SM Definition "Tanner graph"),
 * interleaved with belief-guided local moves of the active checks
 * (Algorithm 1: Evidence test and LocalMove), until the syndrome clears.
 *
 * Conventions for every call:
 *  - Pointers named *_host are host memory; every other buffer is device
 *    memory on the code's device. All arrays are dense, row-major, C order.
 *  - The caller owns every input, output and workspace buffer. The library
 *    owns laim_code, laim_batch_plan and laim_server objects and keeps no
 *    caller pointer after the call's work has completed on its stream.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL is the null stream)
 *    and is asynchronous unless stated otherwise.
 *  - A non-zero status means nothing was enqueued; argument and shape errors
 *    are detected before any work is launched. laim_last_error() returns a
 *    text for the last failing call on the calling thread. No C++ exception
 *    crosses this interface.
 *  - Results depend only on (H, parameters, seed, shot ids, e0): never on
 *    the stream, the batch a shot is in, its position, the launch shape or
 *    the form used.
 */
#ifndef LAIM_H
#define LAIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t laim_status;
#define LAIM_OK 0
#define LAIM_EINVAL (-1) /* bad argument or shape */
#define LAIM_ENOMEM (-2) /* allocation failed or workspace too small */
#define LAIM_EHIP (-3)   /* a HIP runtime call failed */
#define LAIM_EUNSUP (-4) /* valid, but not supported by this library */
#define LAIM_EBUSY (-5)  /* resource exhausted (server slots, budget) */

typedef void* laim_stream; /* hipStream_t */

/* Text of the last failure on this thread ("" if none). */
const char* laim_last_error(void);
/* ABI version of this library (increments on incompatible change). */
int32_t laim_version(void);

/* ------------------------------------------------------------------ codes
 * laim_build_tanner -- the Tanner graph of H (SM Definition "Tanner
 * graph": an edge {v, c} for every H[c][v] = 1) laid out for the device, and
 * the logical basis used by the success test (Preliminaries, conditions (1)
 * and (2)).
 *   m, n             H is m x n (checks x qubits), m, n >= 1.
 *   h_rowptr_host    [m+1] CSR row pointers of H, h_rowptr[0] = 0.
 *   h_col_host       [nnz] column indices; strictly ascending within a row,
 *                    0 <= col < n. Every qubit must lie in >= 1 check.
 *   mg, g_*_host     G (mg x n): the commuting stabilisers whose row space is
 *                    the trivial class (H_Z for Z noise). mg may be 0.
 *                    H G^T = 0 is required (checked).
 *   device           HIP device index that will hold the code.
 *   out              receives the code object (free with laim_free_code).
 * The logical basis (k rows spanning ker(G) modulo row(H)) is computed by
 * GF(2) elimination, which is done for n <= 20480; larger codes must pass
 * their logicals through laim_build_tanner_ex. Check degree <= 32 and qubit
 * degree <= 16 are supported.
 */
typedef struct laim_code laim_code;

laim_status laim_build_tanner(int32_t m, int32_t n, const int32_t* h_rowptr_host,
                              const int32_t* h_col_host, int32_t mg,
                              const int32_t* g_rowptr_host, const int32_t* g_col_host,
                              int32_t device, laim_code** out);

/* As laim_build_tanner, with the logical basis given by the caller: kl rows
 * (CSR, ascending columns), each of even overlap with every row of G
 * (checked) and independent modulo row(H) (not checked). kl = -1 asks for
 * the elimination. */
laim_status laim_build_tanner_ex(int32_t m, int32_t n, const int32_t* h_rowptr_host,
                                 const int32_t* h_col_host, int32_t mg,
                                 const int32_t* g_rowptr_host, const int32_t* g_col_host,
                                 int32_t kl, const int32_t* l_rowptr_host,
                                 const int32_t* l_col_host, int32_t device, laim_code** out);

void laim_free_code(laim_code* code);

/* Sizes: m checks, n qubits, E edges, k logicals, largest check and qubit
 * degree. Any output pointer may be NULL. */
laim_status laim_code_info(const laim_code* code, int32_t* m, int32_t* n, int32_t* E, int32_t* k,
                           int32_t* dc_max, int32_t* dv_max);

/* The logical basis as a dense k x n 0/1 host matrix (out_host [k][n]). */
laim_status laim_code_logicals(const laim_code* code, uint8_t* out_host);

/* Host-only GF(2) elimination (no device involved): writes up to kmax rows
 * of a basis of ker(G) modulo row(H) to out_host [kmax][n] and its size to
 * *k_out. Same limits as laim_build_tanner. */
laim_status laim_host_logicals(int32_t m, int32_t n, const int32_t* h_rowptr_host,
                               const int32_t* h_col_host, int32_t mg, const int32_t* g_rowptr_host,
                               const int32_t* g_col_host, int32_t kmax, uint8_t* out_host,
                               int32_t* k_out);

/* ------------------------------------------------------------------ noise
 * laim_sample_noise -- i.i.d. Bernoulli(p) Z errors (Preliminaries; SM
 * prior). e_out[i][v] = 1 iff w < floor(p 2^32) (p >= 1: always), where w is
 * word (v mod 4) of Philox4x32-10 (Salmon et al., SC'11) with key = seed and
 * counter = (shot_lo, shot_hi, floor(v / 4), 0), shot = shot0 + i.
 *   e_out   device [nshots][n] uint8, written with 0/1.
 * nshots >= 0; p in [0, 1] (values outside are clamped to it).
 */
laim_status laim_sample_noise(const laim_code* code, double p, uint64_t seed, uint64_t shot0,
                              int32_t nshots, uint8_t* e_out, laim_stream stream);

/* laim_syndrome -- s = H e mod 2 (SM, syndrome of an error).
 *   e      device [nshots][n] uint8 (only bit 0 is read)
 *   s_out  device [nshots][m] uint8 */
laim_status laim_syndrome(const laim_code* code, const uint8_t* e, int32_t nshots, uint8_t* s_out,
                          laim_stream stream);

/* ----------------------------------------------------------------- decode
 * Parameters of the round-discretised machine (Algorithm 1 run in rounds):
 * each round runs `iters` BP sweeps (check phase, then qubit phase; BP-LLR2
 * then BP-LLR1; messages start at 0 and are never reset), then every
 * active check whose Poisson clock rang in the round (probability
 * mask_density, word 0 of Philox(key = seed, counter = (shot_lo, shot_hi, c,
 * 16 r + 1)) below floor(mask_density 2^32)) and whose Evidence holds
 * (max over v in N(c) of L_v >= -log(d_c - 1), i.e. Pr_BP >= 1/d_c) flips its
 * LocalMove qubit (the largest belief; ties, compared with ==, broken by
 * word 1 of the same Philox output as tie number floor(w1 ntie / 2^32) in
 * ascending qubit order). A qubit chosen by several checks flips once. The
 * syndrome is then updated (s ^= H f). All arithmetic is FP32 without
 * contraction: every LLR (messages and beliefs) is clamped to [-clamp,
 * clamp] (SM numerical details: CLAMP).
 */
typedef struct {
  int32_t bp;           /* 0: normalised min-sum (alpha * min, sign product); 1: sum-product
                           (BP-LLR2 in box-plus form: output j of a check is F(j-1) [+] B(j+1),
                           with the ascending prefix folds F(k) = F(k-1) [+] m(k) and the
                           descending suffix folds B(k) = m(k) [+] B(k+1) of its inputs m(0..d-1);
                           an empty side is dropped) */
  float alpha;          /* min-sum scale, > 0 (0.75) */
  double q;             /* decoder prior in (0, 1): pi = log(q / (1 - q)) (Table S1: 0.05) */
  float clamp;          /* CLAMP > 0 (Table S1: 1000) */
  int32_t iters;        /* BP sweeps per round, >= 0 (20) */
  int32_t rounds;       /* feedback rounds R, >= 0; a shot not clear after R rounds fails */
  double mask_density;  /* probability that a check's clock rings in a round (0.5) */
  int32_t gauge;        /* must be 0 (the LLR switch of the bit-centric machine is not
                           part of the check-centric machine) */
  int32_t evidence;     /* 1: apply the Evidence test; 0: ablation without it */
  int32_t retire;       /* 1: stop a shot at its first clear syndrome (same z, s, t_clr) */
  uint64_t seed;        /* Philox key for the clocks and tie-breaks */
  int32_t conflict;     /* how one round's move requests combine, LAIM_CONFLICT_* (0: OR) */
  int32_t skip_fixed;   /* 1: skip sweeps that cannot change anything (see below); 0: run all */
  int32_t move;         /* the local move of an acting check, LAIM_MOVE_* (0: LocalMove) */
} laim_decode_params;

/* Local moves. Algorithm 1's LocalMove flips one qubit of an acting check;
 * the LDPC-codes section also names a multi-qubit flip akin to small-set
 * flip, guided by the local beliefs, without a rule for it. The rule here:
 *   SINGLE  the LocalMove qubit (largest belief, random tie-break);
 *   MULTI   every qubit v of N(c) with L_v > 0, i.e. Pr_BP(e_v = 1 | s) > 1/2;
 *           the LocalMove qubit when there is none.
 * Every qubit of a multi-qubit move is one request under the conflict rule
 * (OR or XOR; the sequential rule takes single moves only: LAIM_EUNSUP). */
#define LAIM_MOVE_SINGLE 0
#define LAIM_MOVE_MULTI 1

/* skip_fixed. Within a round the sweep is a fixed map of the messages (the
 * syndrome, prior and parameters do not change), so once a sweep writes
 * every message of a shot back bit for bit, every later sweep does the same
 * until a flip changes the syndrome. With skip_fixed = 1 the resident form
 * detects such a sweep -- sweep i of a round with i = 7 mod 8, and the
 * round's last, compare each new message with the one it replaces -- and
 * leaves the shot's messages as they are for the rest of the round and for
 * following rounds without a flip. A shot's first sweep
 * (v->c messages 0) is a different map and never counts. z, s, t_clr and
 * the beliefs are bit-identical to running every sweep; only the sweeps
 * computed (sweeps_out) differ. The stream form compares on the same
 * sweeps (reading each compared message once more) and skips a 256-shot
 * tile's sweep when every shot of the tile is retired or at a fixed point.
 * Both forms also stop a shot whose messages are at a fixed point at the
 * feedback step while no active check passes Evidence: nothing can change
 * in any later round, so its outputs are final. */

/* Conflict rules. Algorithm 1 lets one clock ring at a time; a round of the
 * discretised machine gathers the requests of every check that rang, and
 * these values say how they combine:
 *   OR          a qubit requested by one or more checks flips once (default);
 *   XOR         a qubit flips once per request, so two requests cancel;
 *   SEQUENTIAL  requests apply one at a time in the order of their ring
 *               times within the round (word 2 of the check's Philox output
 *               for the round, ties by ascending check index), each only if
 *               its check is still active after the requests applied before
 *               it. Beliefs, Evidence and the chosen qubits are those of the
 *               round's start under every rule. */
#define LAIM_CONFLICT_OR 0
#define LAIM_CONFLICT_XOR 1
#define LAIM_CONFLICT_SEQUENTIAL 2

/* Execution forms of laim_decode_rounds; all give identical results. */
#define LAIM_FORM_AUTO 0     /* resident if the code fits in LDS (and, for min-sum,
                                alpha <= 1), else stream */
#define LAIM_FORM_RESIDENT 1 /* one persistent launch, per-shot state in LDS/registers */
#define LAIM_FORM_STREAM 2   /* messages in HBM, one launch per BP sweep and per phase */

/* Workspace needed by laim_decode_rounds for nshots shots in `form`; 0 for
 * bad arguments or a form the code cannot run in. */
size_t laim_workspace_bytes(const laim_code* code, const laim_decode_params* params,
                            int32_t nshots, int32_t form);

/* laim_decode_rounds -- run the machine on nshots shots (ids shot0 + i).
 *   e0         device [nshots][n] uint8: the initial errors (bit 0 read)
 *   workspace  device, >= laim_workspace_bytes(...) bytes, 256-byte aligned;
 *              scratch owned by the caller, contents undefined afterwards
 *   z_out      device [nshots][n] uint8: cumulative correction z
 *   s_out      device [nshots][m] uint8: final syndrome H (e0 ^ z)
 *   tclr_out   device [nshots] int32: rounds completed when the syndrome first
 *              became 0 (0 if H e0 = 0), or -1 if it never did within R
 *   L_out      device [nshots][n] float or NULL: beliefs of the final message
 *              state, clamp(pi + sum over N(v) of m_{c->v}) (for a retired
 *              shot, the state at retirement)
 *   sweeps_out device [nshots] int32 or NULL: BP sweeps computed for each
 *              shot; iters x (rounds the shot ran) unless skip_fixed skipped
 *              some (saturates at 2^31 - 1). The stream form sweeps whole
 *              tiles and reports the method's count, iters x (rounds until
 *              the shot cleared, or R when it did not or retire is 0)
 *   fail_out   device [nshots] uint8 or NULL: the decoder failure of each
 *              shot, exactly as laim_logical_failure(e0, z_out) gives it; the
 *              resident form computes it inside the launch (codes with at
 *              most 128 logicals), otherwise a failure kernel follows
 * Errors: LAIM_EINVAL for bad arguments or an unknown form; LAIM_EUNSUP for
 * form = LAIM_FORM_RESIDENT when the code cannot run in it (a shot's state
 * larger than the LDS, degrees beyond the compiled variants, or min-sum with
 * alpha > 1), and for fail_out on codes with more than 2048 logicals;
 * LAIM_ENOMEM for a workspace smaller than laim_workspace_bytes gives. All
 * are reported before anything is launched.
 * Concurrent calls on different streams may share a laim_code but not a
 * workspace.
 */
laim_status laim_decode_rounds(const laim_code* code, const laim_decode_params* params,
                               const uint8_t* e0, uint64_t shot0, int32_t nshots, void* workspace,
                               size_t ws_bytes, uint8_t* z_out, uint8_t* s_out, int32_t* tclr_out,
                               float* L_out, int32_t* sweeps_out, uint8_t* fail_out, int32_t form,
                               laim_stream stream);

/* Launch shape of the resident form (0 in a field means: choose). */
typedef struct {
  int32_t threads_per_shot; /* threads cooperating on one shot */
  int32_t checks_per_thread;
  int32_t shots_per_block;
} laim_resident_cfg;

/* As laim_decode_rounds in the resident form with an explicit launch shape
 * (used by the autotuner; results do not depend on the shape). */
laim_status laim_decode_rounds_cfg(const laim_code* code, const laim_decode_params* params,
                                   const uint8_t* e0, uint64_t shot0, int32_t nshots,
                                   void* workspace, size_t ws_bytes, uint8_t* z_out,
                                   uint8_t* s_out, int32_t* tclr_out, float* L_out,
                                   int32_t* sweeps_out, uint8_t* fail_out,
                                   const laim_resident_cfg* cfg, laim_stream stream);

/* Size of the static scratch of laim_decode_rounds_static, per device. */
#define LAIM_STATIC_SCRATCH_BYTES (32u << 20)

/* laim_decode_rounds_static -- laim_decode_rounds without a workspace, for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation. The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine); the scratch
 * the chosen form needs -- 256 bytes for the resident form's shot queue, or
 * laim_workspace_bytes(code, params, nshots, LAIM_FORM_STREAM) for the stream
 * form -- comes from a static device array of LAIM_STATIC_SCRATCH_BYTES
 * that each device the library runs on holds until the process ends.
 * Arguments, outputs and results are those of laim_decode_rounds.
 * Errors: as laim_decode_rounds; LAIM_ENOMEM (before anything is launched)
 * when the form needs more scratch than LAIM_STATIC_SCRATCH_BYTES.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents (each call clears what must start at zero): calls that
 * overlap on one device -- on different streams or from different threads
 * -- race and must be serialised by the caller. */
laim_status laim_decode_rounds_static(const laim_code* code, const laim_decode_params* params,
                                      const uint8_t* e0, uint64_t shot0, int32_t nshots,
                                      uint8_t* z_out, uint8_t* s_out, int32_t* tclr_out,
                                      float* L_out, int32_t* sweeps_out, uint8_t* fail_out,
                                      int32_t form, laim_stream stream);

/* laim_resident_variant -- the resident kernel laim_decode_rounds (or, with
 * cfg, laim_decode_rounds_cfg) would run for these parameters: its template
 * degrees, checks per thread, and whether it is the tiled variant. The tiled
 * variant runs min-sum on the 2D toric layout (checks i L + j, L a multiple
 * of 4, each sharing one qubit with each lattice neighbour) with 8 checks per
 * thread and m / 8 threads per shot: each thread's checks form a 2 x 4 tile,
 * and the messages on the 10 qubits inside a tile stay in the thread's
 * registers through a round's sweeps. Results never depend on the variant.
 * Any output pointer may be NULL. Errors: LAIM_EUNSUP when the code or the
 * parameters cannot run in the resident form; LAIM_EINVAL for bad
 * arguments. */
laim_status laim_resident_variant(const laim_code* code, const laim_decode_params* params,
                                  const laim_resident_cfg* cfg, int32_t* dc, int32_t* dv,
                                  int32_t* checks_per_thread, int32_t* tiled);

/* Sets the resident launch shape used from now on for this code and BP
 * rule (the autotuner's choice); cfg = NULL restores the built-in rule:
 * min-sum on the 2D toric layout takes the tiled variant (8 checks per
 * thread, m / 8 threads per shot, blocks near 128 threads with wavefronts at
 * least 80% full); otherwise 1, 2, 4 or 8 checks per thread for m up to 256,
 * 512, 1024 and beyond, and 256-thread blocks. A field given as 0 in cfg is
 * chosen by the same rule. */
laim_status laim_set_resident_cfg(laim_code* code, int32_t bp, const laim_resident_cfg* cfg);
/* The launch shape that would be used (after the built-in rule). */
laim_status laim_get_resident_cfg(const laim_code* code, int32_t bp, laim_resident_cfg* cfg);

/* laim_logical_failure -- decoder failure (Preliminaries): with r = e0 ^ z,
 * fail = [H r != 0] or [r not in row(G)], the latter tested as any odd
 * overlap of r with a row of the logical basis.
 *   e0, z     device [nshots][n] uint8
 *   fail_out  device [nshots] uint8 (0/1) */
laim_status laim_logical_failure(const laim_code* code, const uint8_t* e0, const uint8_t* z,
                                 int32_t nshots, uint8_t* fail_out, laim_stream stream);

/* ------------------------------------------------- continuous-time machine
 * Algorithm 1 as stated: BP relaxes by tau dm/dt = F_BP(m; S) - m while
 * unit-rate Poisson clocks ring at the checks (SM numerical details: Euler
 * steps of dt, waiting times ~ Exp(|S|), Table S1's dt, tau, t_max).
 * One Euler step updates both message directions from the state before it
 * (Jacobi form): m <- clamp(m + lambda (F - m)) with lambda = (float)(dt / tau),
 * F_{c->v} by BP-LLR2 and F_{v->c} = clamp(pi + sum over N(v)\c of m_{c'->v})
 * by BP-LLR1; all messages start at 0.
 * Events: event j draws Philox(key = seed, counter = (shot_lo, shot_hi, j, 2))
 * = (w0, w1, w2, w3). Its time is the previous event's (0 for j = 0) plus
 * -ln((w0 + 1) 2^-32) / |S| in double precision (|S| = active checks after
 * the previous event); the ringing check is active check number
 * floor(w1 |S| / 2^32) in ascending order; if its Evidence holds (as in the
 * round machine) it flips its LocalMove qubit, ties broken by w2. An event
 * at time T acts on the BP state after floor(T / dt) Euler steps; events due
 * at the same step act in order.
 */
typedef struct {
  int32_t bp;       /* 0: normalised min-sum, 1: sum-product (as laim_decode_params) */
  float alpha;      /* min-sum scale, > 0 */
  double q;         /* decoder prior in (0, 1) */
  float clamp;      /* CLAMP > 0 */
  double dt;        /* Euler step in clock units, > 0 (Table S1: 0.001 or 0.01) */
  double tau;       /* relaxation time, > 0 (Table S1: 0.1) */
  double t_max;     /* a shot not clear by t_max fails; the run makes floor(t_max / dt + 1/2)
                       Euler steps at most (t_max / dt <= 2^31 - 1) */
  int32_t evidence; /* 1: apply the Evidence test */
  uint64_t seed;    /* Philox key for the clocks and tie-breaks */
  int32_t skip_fixed; /* 1: skip Euler steps that cannot change the messages. Between
                         moves the step is a fixed map of the messages; once one
                         leaves every message bit for bit as it was (tested 7 steps
                         after the start and after each move, then at intervals that
                         double from 8 to 256 while the messages keep changing), the
                         steps up to the next event are skipped.
                         Events are still handled one by one: all outputs, counts
                         included, equal those of every step. 0: run every step. */
} laim_continuous_params;

/* Workspace of laim_decode_continuous (the shot queue), in bytes. */
#define LAIM_CONTINUOUS_WORKSPACE_BYTES 256

/* laim_decode_continuous -- the continuous-time machine on nshots shots
 * (ids shot0 + i), one resident block per shot at a time.
 *   e0         device [nshots][n] uint8: the initial errors (bit 0 read)
 *   workspace  device, >= LAIM_CONTINUOUS_WORKSPACE_BYTES, 256-byte aligned
 *   z_out      device [nshots][n] uint8: cumulative correction z
 *   s_out      device [nshots][m] uint8: final syndrome H (e0 ^ z)
 *   tclr_out   device [nshots] double: time of the event that cleared the
 *              syndrome (0 if H e0 = 0), or -1 if it did not clear by t_max
 *   counts_out device [nshots][2] int32 or NULL: events (clock rings of
 *              active checks) and moves (flips) of each shot
 *   steps_out  device [nshots] int32 or NULL: Euler steps computed for each
 *              shot; every step of the run unless skip_fixed skipped some
 *   fail_out   device [nshots] uint8 or NULL: logical failure, as
 *              laim_logical_failure
 *   checks_per_thread  0 to choose, else 1, 2, 4 or 8 (a launch shape;
 *              results do not depend on it)
 * Errors: LAIM_EINVAL for bad arguments, LAIM_EUNSUP for codes with check
 * degree > 8 or qubit degree > 4 or too large for LDS, LAIM_ENOMEM for a
 * short workspace; nothing is written then.
 */
laim_status laim_decode_continuous(const laim_code* code, const laim_continuous_params* params,
                                   const uint8_t* e0, uint64_t shot0, int32_t nshots,
                                   void* workspace, size_t ws_bytes, uint8_t* z_out, uint8_t* s_out,
                                   double* tclr_out, int32_t* counts_out, int32_t* steps_out,
                                   uint8_t* fail_out, int32_t checks_per_thread, laim_stream stream);

/* --------------------------------------------------- bit-centric machine
 * The discrete bit-centric machine of the SM ("Setup and algorithm") for
 * codes whose checks all have degree 2 (the repetition code). No randomness:
 * iteration i updates, from the state of iteration i - 1 (Jacobi),
 *   m_{c->v} = (-1)^{s_c} m_{w->c} (w the other bit of c; BP-LLR2, d_c = 2),
 *   m_{v->c} = pi_v + sum over c' in N(v)\c of m_{c'->v} (BP-LLR1),
 *   L_v = pi_v + sum over N(v) of m_{c->v} (ascending c),
 * flips f_v = [L_v > 0], updates s ^= H f and negates pi_v and the new
 * messages of flipped bits (the LLR switch). Double precision; messages
 * start at 0, pi_v at log(q / (1 - q)).
 */
/* laim_decode_bitcentric -- `iters` iterations on each of nshots shots.
 *   e0        device [nshots][n] uint8: the initial errors
 *   z_out     device [nshots][n] uint8: cumulative flips z (error e0 ^ z)
 *   iclr_out  device [nshots] int32: first iteration after which s = 0
 *             (0 if H e0 = 0, -1 if never within iters)
 *   L_out     device [nshots][n] double or NULL: beliefs of the last iteration
 * Errors: LAIM_EUNSUP unless every check has degree 2 and every bit degree
 * <= 4, n and m <= 3072 and the state fits in LDS; LAIM_EINVAL for bad arguments.
 */
laim_status laim_decode_bitcentric(const laim_code* code, double q, const uint8_t* e0,
                                   int32_t nshots, int32_t iters, uint8_t* z_out, int32_t* iclr_out,
                                   double* L_out, laim_stream stream);

/* Forms of the bit-centric machine; both give the same results bit for bit.
 * The chain form takes chains (checks {v, v + 1}, plus {0, n - 1} when
 * periodic) of 2 to 1008 bits (3 to 1024 periodic) in which no bit other than
 * bit 0 has its left check at the larger index: one wavefront per shot with
 * each bit's messages in its lane's registers, run in the frame of the
 * current error e0 ^ z (where the syndrome signs and the LLR switch cancel
 * and each iteration shifts the messages one bit along the chain and adds
 * the prior). The block form takes any code the call above accepts: one
 * workgroup per shot with the messages in LDS. */
#define LAIM_BC_AUTO 0  /* the chain form where it applies, else the block form */
#define LAIM_BC_CHAIN 1
#define LAIM_BC_BLOCK 2

/* laim_decode_bitcentric_form -- laim_decode_bitcentric in `form`.
 * Errors: as laim_decode_bitcentric; LAIM_EUNSUP for form = LAIM_BC_CHAIN
 * on a code the chain form does not take; LAIM_EINVAL for an unknown form. */
laim_status laim_decode_bitcentric_form(const laim_code* code, double q, const uint8_t* e0,
                                        int32_t nshots, int32_t iters, int32_t form, uint8_t* z_out,
                                        int32_t* iclr_out, double* L_out, laim_stream stream);

/* -------------------------------------------------------- online decoding
 * Online decoding (Discussion: faults and syndrome rounds keep arriving; the
 * Tanner graph is promoted to a spacetime decoding graph and the local
 * dynamics runs in overlapping spacetime windows). The paper fixes neither
 * the noise nor the window rule; this library's:
 *  - N syndrome rounds t = 1..N. Before round t each qubit gets a new Z
 *    error e_t[v] ~ Bernoulli(p): word (v mod 4) of Philox(key = seed,
 *    counter = (shot_lo, shot_hi, floor(v / 4), 16 t + 3)) below
 *    floor(p 2^32). Round t measures H E_t ^ eps_t, E_t = e_1 ^ ... ^ e_t,
 *    with measurement errors eps_t[c] ~ Bernoulli(p_meas) (word (c mod 4)
 *    of Philox(seed, (shot_lo, shot_hi, floor(c / 4), 16 t + 4))); the last
 *    round is perfect (eps_N = 0). seed is the decode parameters' seed.
 *  - Detectors D_t = H e_t ^ eps_t ^ eps_{t-1} (eps_0 = 0).
 *  - A window of w rounds is the code whose variables are the data errors
 *    (tau, v) -> tau n + v and the measurement errors (tau, c) ->
 *    w n + tau m + c of its rounds (not of a final perfect round), and whose
 *    check tau m + c is detector (tau, c).
 *  - Window k covers rounds k C + 1 .. min(k C + W, N); the last window is
 *    the first that reaches N. Its syndrome is its rounds' detectors, with
 *    the measurement corrections committed for round k C added to its
 *    first round; the round machine (laim_decode_params, R = rounds per
 *    window) decodes it from fresh messages, its rounds numbered from k R
 *    for the clocks. Its first C rounds (every round, in the last window)
 *    are committed: their data corrections add to z, and the measurement
 *    corrections of its last committed round carry into the next window.
 *  - Failure is the offline test (laim_logical_failure) on E_N and z.
 */
typedef struct {
  int32_t rounds_total; /* N syndrome rounds (>= 1), the last one perfect */
  int32_t window;       /* W rounds per window (>= 1) */
  int32_t commit;       /* C rounds committed per window, 1 <= C <= W */
  double p;             /* data error rate per qubit and round */
  double p_meas;        /* measurement error rate per check and round */
} laim_online_params;

typedef struct laim_online_plan laim_online_plan;

/* Builds the window codes of `code` for these parameters on the code's
 * device (the plan keeps a pointer to code, which must outlive it). */
laim_status laim_online_plan_create(const laim_code* code, const laim_online_params* op,
                                    laim_online_plan** out);
void laim_online_plan_destroy(laim_online_plan* plan);
/* Workspace of laim_decode_online for nshots shots (0 for bad arguments). */
size_t laim_online_workspace_bytes(const laim_online_plan* plan, const laim_decode_params* params,
                                   int32_t nshots);
/* laim_decode_online -- online decode of nshots shots (ids shot0 + i), all
 * shots advancing window by window.
 *   e_in, eps_in  device [nshots][N][n] and [nshots][N][m] uint8, or both
 *                 NULL: the errors to use instead of sampled ones (the last
 *                 round's eps_in is ignored: that round is perfect)
 *   workspace     device, >= laim_online_workspace_bytes, 256-byte aligned
 *   z_out         device [nshots][n]: the committed data correction
 *   E_out         device [nshots][n] or NULL: the final error E_N
 *   fail_out      device [nshots] or NULL: failure of (E_N, z)
 *   cleared_out   device [nshots] int32 or NULL: windows whose syndrome cleared
 * Errors: LAIM_EINVAL for bad arguments, LAIM_ENOMEM for a short workspace,
 * as laim_decode_rounds for the parameters; nothing is launched then. */
laim_status laim_decode_online(const laim_online_plan* plan, const laim_decode_params* params,
                               uint64_t shot0, int32_t nshots, const uint8_t* e_in,
                               const uint8_t* eps_in, void* workspace, size_t ws_bytes,
                               uint8_t* z_out, uint8_t* E_out, uint8_t* fail_out,
                               int32_t* cleared_out, laim_stream stream);

/* ----------------------------------------------------------- batched form
 * One persistent launch over shots of several codes and sizes (each item a
 * contiguous range of shot ids of one code with its own parameters and
 * outputs, laid out as in laim_decode_rounds). The plan precomputes the work
 * list, owns its device workspace and records the launch sequence in a HIP
 * graph that laim_batch_plan_launch replays. Inputs and outputs are read and
 * written at the addresses given at creation. Items whose code cannot run in
 * the resident form (a shot's state larger than the LDS, degrees beyond the
 * compiled variants, or min-sum with alpha > 1) run in the stream form,
 * recorded in the same graph after the persistent launch; the plan owns
 * their HBM workspace. Results never depend on which form an item takes.
 */
typedef struct {
  const laim_code* code;
  laim_decode_params params;
  const uint8_t* e0;  /* device [nshots][n] */
  uint64_t shot0;
  int32_t nshots;
  uint8_t* z_out;     /* device [nshots][n] */
  uint8_t* s_out;     /* device [nshots][m] */
  int32_t* tclr_out;  /* device [nshots] */
  uint8_t* fail_out;  /* device [nshots] or NULL: logical failure of each shot */
} laim_batch_item;

typedef struct laim_batch_plan laim_batch_plan;

laim_status laim_batch_plan_create(const laim_batch_item* items, int32_t nitems,
                                   laim_stream stream, laim_batch_plan** out);
laim_status laim_batch_plan_launch(laim_batch_plan* plan, laim_stream stream);
void laim_batch_plan_destroy(laim_batch_plan* plan);

/* --------------------------------------------------------------- serving
 * A continuous-batching server: requests (one shot of one code each, with
 * its own rounds budget) are admitted while device memory and slots allow,
 * keep their BP messages and syndrome state resident in device memory
 * across rounds, and advance one round per laim_server_step together with
 * every other resident request. Requests that do not fit wait in FIFO order.
 * Calls on one server must not overlap; the server uses its own stream.
 */
typedef struct laim_server laim_server;

typedef struct {
  uint64_t ticket;     /* from laim_server_submit */
  int32_t round;       /* rounds completed by this request after this step */
  int32_t done;        /* 1 when the request finished: cleared and retired, rounds exhausted, or
                          frozen (with skip_fixed: its messages at a fixed point, nothing flipped
                          and no active check passing Evidence, so no later round can change
                          its result) */
  int32_t tclr;        /* as in laim_decode_rounds (-1 while not cleared) */
  int32_t flips;       /* qubits flipped in this round */
  int32_t defects;     /* syndrome weight after this round */
  int32_t fail;        /* decoder failure of the current state (final when done) */
  int64_t latency_ns;  /* this round: from its input being ready (submission for round 0,
                          the previous round's completion otherwise) to its results on the host */
} laim_server_event;

/* Creates a server on `device` with a device-memory budget for request
 * state (per request about n + 4 m d_c + n + m + 256 bytes, 256-aligned
 * parts) and at most max_slots requests advanced per step. Requests must
 * use codes with check degree <= 8 and qubit degree <= 4 (min-sum with
 * alpha <= 1). */
laim_status laim_server_create(int32_t device, size_t mem_budget_bytes, int32_t max_slots,
                               laim_server** out);
/* Queues one request for shot `shot_id` and returns a ticket. The request's
 * initial error (the hidden error of the problem statement, Preliminaries)
 * is either given or drawn on the device:
 *   e0_host  [n] host 0/1 values, copied before the call returns; or NULL:
 *            the error is sampled on the device at admission from (key =
 *            params->seed, shot id, p), exactly as laim_sample_noise(code, p,
 *            params->seed, shot_id, 1) draws it (i.i.d. Bernoulli(p) Z errors).
 *   p        noise rate of a sampled error, used only when e0_host is NULL
 *            (values outside [0, 1] are clamped to it; NaN is an error).
 * A request with params->rounds = 0 runs no round: its first step reports the
 * start state (t_clr 0 if H e0 = 0, else -1) and finishes it.
 * Errors: LAIM_EINVAL for bad arguments, LAIM_EUNSUP for a code the server
 * cannot run, LAIM_ENOMEM when one request of this code needs more device
 * state than the server's whole budget (it could never be admitted). */
laim_status laim_server_submit(laim_server* srv, const laim_code* code,
                               const laim_decode_params* params, uint64_t shot_id,
                               const uint8_t* e0_host, double p, uint64_t* ticket);
/* Admits waiting requests that fit, advances resident requests by one round
 * -- at most max_events of them, the oldest first -- and returns one event per
 * advanced request (blocking until the round's results are on the host).
 * events_host has room for max_events; requests beyond it wait for a later
 * step, so that every finished request reports its done event. */
laim_status laim_server_step(laim_server* srv, laim_server_event* events_host, int32_t max_events,
                             int32_t* n_events);
/* Final z [n], s [m] and t_clr of a finished request (host copies); the
 * request's storage is released afterwards. */
laim_status laim_server_result(laim_server* srv, uint64_t ticket, uint8_t* z_host, uint8_t* s_host,
                               int32_t* tclr);
/* Resident requests, waiting requests, bytes in use. */
laim_status laim_server_stats(const laim_server* srv, int32_t* resident, int32_t* waiting,
                              size_t* bytes_in_use);
void laim_server_destroy(laim_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* LAIM_H */
