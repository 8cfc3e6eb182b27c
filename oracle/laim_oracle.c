/*
 * laim_oracle.c -- CPU oracle for the local autonomous inference machine.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
 * loads this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do. It shares no code with the HIP path: every
 * routine here (Philox, the FP32 transcendental functions, BP, the feedback
 * rule, GF(2) elimination) is written separately from the paper and from the
 * published definitions it names.
 *
 * What it computes (the paper's sections are cited per function):
 *   - i.i.d. Bernoulli(p) Z errors from a counter-based generator
 *     (Preliminaries; SM "Tanner graphs ..." prior),
 *   - the syndrome s = H e (SM, syndrome definition),
 *   - BP in LLR form, Eqs. (BP-LLR1) and (BP-LLR2), either sum-product as
 *     printed or normalised min-sum (a reading: the paper uses sum-product),
 *   - the round-discretised check-centric machine of Algorithm 1: BP, then
 *     every active check whose clock rang this round tests Evidence and
 *     flips the argmax qubit (LocalMove) -- or, as the multi-qubit move the
 *     LDPC-codes section mentions, every qubit of the check whose belief is
 *     positive -- then the syndrome update; the round's move requests
 *     combine by one of three conflict rules,
 *   - the decoding-success test (Preliminaries, conditions (1) and (2)) by an
 *     independent GF(2) rank test,
 *   - the continuous-time machine of Algorithm 1 as stated: Euler-damped
 *     BP and Poisson clock events (SM "Numerical details"),
 *   - for pins only: the discrete bit-centric machine of the SM ("Setup and
 *     algorithm"), in double precision.
 *
 * Pins (the test suite checks each part against what the paper and the
 * mathematics fix: window and tree closed forms, brute-force marginals,
 * invariants, special cases, the bit-centric theorem). Parity unpinned:
 *   - min-sum and sum-product dynamics, round and continuous, on loopy codes
 *     (toric, bivariate-bicycle, membrane) beyond those invariants and
 *     special cases: only the GPU parity tests compare them;
 *   - the round machine's logical error rates, which the paper does not
 *     print (its dynamics is the continuous one);
 *   - which Philox word gives the sequential conflict rule its ring times;
 *   - the rule of the multi-qubit move (a reading; the paper names such moves
 *     without specifying them): beyond its reduction to LocalMove and the
 *     replay of its decisions, only the GPU parity tests compare it.
 *
 * Precision: the decoder runs in FP32 because its integer decisions (which
 * check moves, which qubit flips) are taken from FP32 messages; every float
 * expression is evaluated left to right, one rounding per operation; the
 * file must be compiled with -ffp-contract=off and without fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_VERSION 2

int orc_version(void) { return ORC_VERSION; }

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------
 * Philox4x32-10, as defined by Salmon, Moraes, Dror and Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3" (SC'11): a 4-word counter, 2-word key,
 * ten rounds; each round multiplies words 0 and 2 by the two round
 * multipliers, swaps and xors the high halves with the other words and the
 * round key; the key advances by the two Weyl increments between rounds.
 * ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  const uint32_t MUL0 = 0xD2511F53u, MUL1 = 0xCD9E8D57u;
  const uint32_t WEYL0 = 0x9E3779B9u, WEYL1 = 0xBB67AE85u;
  uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += WEYL0;
      k1 += WEYL1;
    }
    uint64_t p0 = (uint64_t)MUL0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)MUL1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Bernoulli(p) from one uniform 32-bit word w: the event w < floor(p * 2^32)
 * (p >= 1: always; p <= 0: never). Returned as a 64-bit bound so p = 1 is
 * representable. */
uint64_t orc_bernoulli_bound(double p) {
  if (!(p > 0.0)) return 0;
  if (p >= 1.0) return (uint64_t)1 << 32;
  return (uint64_t)floor(p * 4294967296.0);
}

static void philox_for(uint64_t seed, uint64_t shot, uint32_t w2, uint32_t w3, uint32_t out[4]) {
  uint32_t ctr[4] = {(uint32_t)shot, (uint32_t)(shot >> 32), w2, w3};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------
 * FP32 evaluation of the sum-product check rule (BP-LLR2).
 *
 * 2 atanh(prod tanh(m_i / 2)) is evaluated as the pairwise "box-plus" fold
 * of the incoming LLRs (Hagenauer, Offer and Papke, IEEE Trans. Inf. Theory
 * 42 (1996)), using the exact identity
 *   a [+] b := 2 atanh(tanh(a/2) tanh(b/2))
 *            = sg(a) sg(b) [min(|a|, |b|) + g(|a| + |b|) - g(||a| - |b||)],
 *   g(y) := log(1 + e^{-y}),
 * whose correction terms lie in [0, log 2], so no intermediate saturates
 * before the clamp (a literal FP32 tanh product rounds to +-1 once |m| > 17
 * and then jumps to +-CLAMP). +inf is the identity of the fold (an empty
 * product is 1, whose 2 atanh is +inf).
 *
 * g is built from textbook methods with IEEE +, -, *, fused multiply-add
 * (one rounding) and exponent-field manipulation only, so that its result
 * does not depend on the platform:
 * exp: Cody-Waite argument reduction x = k ln2 + r with ln2 split into a
 *   16-significant-bit head (k*head exact for |k| < 256) and a tail, the
 *   degree-7 Taylor polynomial of e^r (coefficients 1/j!) by Horner with a
 *   fused multiply-add per step, then scaling by 2^k through the exponent
 *   field;
 * log(1 + u), u in [0, 1]: u Q(u), Q the degree-9 polynomial interpolating
 *   log(1 + u)/u at the 10 Chebyshev nodes of [0, 1], by Horner with a
 *   fused multiply-add per step.
 * ---------------------------------------------------------------------- */
static float f32_from_bits(uint32_t b) { float f; memcpy(&f, &b, 4); return f; }

/* e^{-a} for a >= 0 (a = +inf allowed). Results below 2^-115 are returned
 * as 0, which keeps every intermediate a normal number. */
float orc_exp_neg(float a) {
  if (!(a <= 80.0f)) return 0.0f; /* also catches +inf */
  const float LN2_HEAD = f32_from_bits(0x3F317200u); /* ln2 with low 8 mantissa bits cleared */
  const float LN2_TAIL = (float)(0.69314718055994530942 - 0.693145751953125);
  const float INV_LN2 = (float)1.44269504088896340736;
  float x = -a;
  float kf = floorf(fmaf(x, INV_LN2, 0.5f));
  float r = fmaf(-kf, LN2_TAIL, fmaf(-kf, LN2_HEAD, x));
  float p = 1.0f / 5040.0f;
  p = fmaf(p, r, 1.0f / 720.0f);
  p = fmaf(p, r, 1.0f / 120.0f);
  p = fmaf(p, r, 1.0f / 24.0f);
  p = fmaf(p, r, 1.0f / 6.0f);
  p = fmaf(p, r, 0.5f);
  p = fmaf(p, r, 1.0f);
  p = fmaf(p, r, 1.0f);
  int k = (int)kf;
  float scale = f32_from_bits((uint32_t)(k + 127) << 23);
  return p * scale;
}

/* log(1 + u) for u in [0, 1] as u Q(u), Q the degree-9 polynomial that
 * interpolates log(1 + u)/u at the 10 Chebyshev nodes of [0, 1] (computed in
 * 40-digit arithmetic, coefficients rounded to FP32), in Horner form with a
 * fused multiply-add per step. No division; relative error below 3 ulp over
 * [0, 1] in FP32. */
float orc_log1p_unit(float u) {
  float q = -0x1.a04acap-9f;
  q = fmaf(q, u, 0x1.402f4cp-6f);
  q = fmaf(q, u, -0x1.cdd008p-5f);
  q = fmaf(q, u, 0x1.afdde8p-4f);
  q = fmaf(q, u, -0x1.38b908p-3f);
  q = fmaf(q, u, 0x1.92b430p-3f);
  q = fmaf(q, u, -0x1.ff0254p-3f);
  q = fmaf(q, u, 0x1.554bd6p-2f);
  q = fmaf(q, u, -0x1.ffffb8p-2f);
  q = fmaf(q, u, 1.0f);
  return u * q;
}

/* g(y) = log(1 + e^{-y}) for y >= 0. */
float orc_softplus_neg(float y) { return orc_log1p_unit(orc_exp_neg(y)); }

/* a [+] b, with sg(x) = -1 if x < 0 else +1, evaluated on magnitudes:
 *   |a| [+] |b| = min(|a|, |b|) + g(|a| + |b|) - g(||a| - |b||) >= 0,
 * (a rounding below zero is set to +0), then the sign sg(a) sg(b) for a
 * nonzero result; a zero result is +0. This makes the FP32 result exactly
 * odd in each argument (up to the sign of zero) and symmetric, and
 * (+inf) [+] x the value of x (+0 for -0). */
float orc_boxplus(float a, float b) {
  float aa = fabsf(a), ab = fabsf(b);
  float mn = (ab < aa) ? ab : aa;
  float diff = (aa < ab) ? (ab - aa) : (aa - ab);
  float mag = (mn + orc_softplus_neg(aa + ab)) - orc_softplus_neg(diff);
  if (mag < 0.0f) mag = 0.0f;
  int neg = (a < 0.0f) ^ (b < 0.0f);
  return (neg && mag > 0.0f) ? -mag : mag;
}

static float clampf_(float x, float C) {
  if (x > C) return C;
  if (x < -C) return -C;
  return x;
}

/* ------------------------------------------------------------------------
 * Tanner graph (SM Definition "Tanner graph"): check c has the qubits
 * N(c) = row c of H (ascending); qubit v has the checks N(v) (ascending).
 * Edges are numbered in row order of H: edge rowptr[c] + j is (c, N(c)[j]).
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t m, n, E;
  const int32_t* rowptr; /* [m+1] */
  const int32_t* col;    /* [E] */
  int32_t* vptr;         /* [n+1] */
  int32_t* vedge;        /* [E]: edges of qubit v, ascending check order */
} tanner;

static int tanner_init(tanner* T, int32_t m, int32_t n, const int32_t* rowptr, const int32_t* col) {
  T->m = m; T->n = n; T->E = rowptr[m];
  T->rowptr = rowptr; T->col = col;
  T->vptr = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  T->vedge = (int32_t*)malloc(sizeof(int32_t) * (size_t)(T->E > 0 ? T->E : 1));
  if (!T->vptr || !T->vedge) return -2;
  for (int32_t e = 0; e < T->E; ++e) T->vptr[col[e] + 1]++;
  for (int32_t v = 0; v < n; ++v) T->vptr[v + 1] += T->vptr[v];
  int32_t* fill = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  if (!fill) return -2;
  for (int32_t c = 0; c < m; ++c) /* ascending c, so each qubit's list is ascending */
    for (int32_t e = rowptr[c]; e < rowptr[c + 1]; ++e) {
      int32_t v = col[e];
      T->vedge[T->vptr[v] + fill[v]++] = e;
    }
  free(fill);
  return 0;
}

static void tanner_free(tanner* T) {
  free(T->vptr);
  free(T->vedge);
}

/* ------------------------------------------------------------------------
 * Noise and syndrome.
 * ---------------------------------------------------------------------- */

/* e[v] = 1[w_v < floor(p 2^32)], w_v = word (v mod 4) of
 * Philox(key = seed, counter = (shot_lo, shot_hi, floor(v/4), 0)). */
void orc_sample_noise(int32_t n, double p, uint64_t seed, uint64_t shot0, int32_t nshots,
                      uint8_t* e_out) {
  uint64_t bound = orc_bernoulli_bound(p);
  for (int32_t i = 0; i < nshots; ++i) {
    uint64_t shot = shot0 + (uint64_t)i;
    for (int32_t v = 0; v < n; ++v) {
      uint32_t w[4];
      philox_for(seed, shot, (uint32_t)(v >> 2), 0u, w);
      e_out[(size_t)i * n + v] = ((uint64_t)w[v & 3] < bound) ? 1 : 0;
    }
  }
}

/* s_c = XOR over v in N(c) of e_v, for nshots rows of e. */
void orc_syndrome(int32_t m, int32_t n, const int32_t* rowptr, const int32_t* col,
                  const uint8_t* e, int32_t nshots, uint8_t* s_out) {
  for (int32_t i = 0; i < nshots; ++i)
    for (int32_t c = 0; c < m; ++c) {
      uint8_t x = 0;
      for (int32_t k = rowptr[c]; k < rowptr[c + 1]; ++k) x ^= e[(size_t)i * n + col[k]] & 1u;
      s_out[(size_t)i * m + c] = x;
    }
}

/* ------------------------------------------------------------------------
 * BP in LLR form.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t bp;            /* 0: normalised min-sum, 1: sum-product (BP-LLR2) */
  float alpha;           /* min-sum normalisation */
  double q;              /* decoder prior; pi = log(q / (1 - q)) */
  float clamp;           /* every LLR is clamped to [-clamp, clamp] */
  int32_t iters;         /* BP iterations per round */
  int32_t rounds;        /* feedback rounds */
  double mask_density;   /* probability that a check's clock rang in a round */
  int32_t gauge;         /* 1: negate pi and messages of flipped qubits */
  int32_t evidence;      /* 1: apply the Evidence test */
  int32_t retire;        /* 1: stop a shot once its syndrome is clear */
  uint64_t seed;
  int32_t conflict;      /* how one round's move requests combine: ORC_CONFLICT_* */
  int32_t move;          /* ORC_MOVE_SINGLE (LocalMove) or ORC_MOVE_MULTI */
} orc_params;

/* Local moves of an acting check (LDPC-codes section: besides the one-qubit
 * LocalMove of Algorithm 1, a multi-qubit flip akin to small-set flip,
 * guided by the local beliefs). The paper gives no rule for the multi-qubit
 * move; the reading here:
 *   SINGLE  the LocalMove qubit: the largest belief in N(c), ties broken at
 *           random (Algorithm 1);
 *   MULTI   every qubit v of N(c) whose belief says it more likely flipped
 *           than not, Pr_BP(e_v = 1 | s) > 1/2, i.e. L_v > 0; if there is
 *           none, the LocalMove qubit. With exactly one such qubit the two
 *           coincide (it is then the unique largest belief). */
enum { ORC_MOVE_SINGLE = 0, ORC_MOVE_MULTI = 1 };

/* Move requests of one round combine (Algorithm 1 has one clock ring at a
 * time; a round gathers several, so a rule is needed):
 *   OR         a qubit requested by at least one check flips once;
 *   XOR        a qubit flips once per request (two requests cancel);
 *   SEQUENTIAL the requests are applied one at a time in the order of their
 *              ring times within the round (word 2 of the check's Philox
 *              output, ties by ascending check index); a request applies
 *              only if its check is still active, i.e. its syndrome bit,
 *              updated by the moves already applied, is 1. */
enum { ORC_CONFLICT_OR = 0, ORC_CONFLICT_XOR = 1, ORC_CONFLICT_SEQUENTIAL = 2 };

/* Check-to-qubit rule (BP-LLR2) for edge j of check c:
 *   m_{c->v} = (-1)^{s_c + d_c} * CN_{w in N(c)\v}(m_{w->c}), then clamped;
 * sum-product: CN = 2 atanh(prod tanh(m/2)), evaluated with box-plus as
 *   F_{j-1} [+] B_{j+1}, F_k = F_{k-1} [+] m_k (F_{-1} = +inf),
 *   B_k = m_k [+] B_{k+1} (B_{d_c} = +inf), an empty side dropped,
 * the prefix and suffix folds of the inputs in ascending order (so all
 * outputs of a check need 3 (d_c - 2) box-plus steps);
 * min-sum:     CN = (alpha * min |m|) * prod sg(m), sg(x) = -1 if x < 0
 *              else +1. An empty product is 1 and an empty minimum is +inf. */
static float check_rule(const orc_params* P, const float* mvc_row, int32_t dc, int32_t j,
                        int32_t s_c) {
  int sigma_neg = (int)((s_c + dc) & 1);
  float out;
  if (P->bp == 1) {
    /* (+inf) [+] x is x (with -0 made +0); an empty side is +inf */
    float F = INFINITY, B = INFINITY;
    for (int32_t i = 0; i < j; ++i) F = orc_boxplus(F, mvc_row[i]);
    for (int32_t i = dc - 1; i > j; --i) B = orc_boxplus(mvc_row[i], B);
    float acc;
    if (j == 0)
      acc = B;
    else if (j == dc - 1)
      acc = F;
    else
      acc = orc_boxplus(F, B);
    out = sigma_neg ? -acc : acc;
  } else {
    float minabs = INFINITY;
    int neg = sigma_neg;
    for (int32_t i = 0; i < dc; ++i) {
      if (i == j) continue;
      float a = fabsf(mvc_row[i]);
      if (a < minabs) minabs = a;
      if (mvc_row[i] < 0.0f) neg ^= 1;
    }
    float mag = P->alpha * minabs;
    out = neg ? -mag : mag;
  }
  return clampf_(out, P->clamp);
}

/* Check phase: every m_{c->v} from the current m_{v->c} and s. */
static void check_phase(const tanner* T, const orc_params* P, const float* mvc, const uint8_t* s,
                        float* mcv) {
  for (int32_t c = 0; c < T->m; ++c) {
    int32_t b = T->rowptr[c], dc = T->rowptr[c + 1] - b;
    for (int32_t j = 0; j < dc; ++j) mcv[b + j] = check_rule(P, mvc + b, dc, j, s[c]);
  }
}

/* Qubit-to-check rule (BP-LLR1): m_{v->c} = pi_v + sum over c' in N(v)\c of
 * m_{c'->v}, added left to right in ascending c', then clamped. */
static void var_phase(const tanner* T, const orc_params* P, const float* pi_v, const float* mcv,
                      float* mvc) {
  for (int32_t v = 0; v < T->n; ++v) {
    int32_t b = T->vptr[v], dv = T->vptr[v + 1] - b;
    for (int32_t j = 0; j < dv; ++j) {
      float acc = pi_v[v];
      for (int32_t i = 0; i < dv; ++i)
        if (i != j) acc = acc + mcv[T->vedge[b + i]];
      mvc[T->vedge[b + j]] = clampf_(acc, P->clamp);
    }
  }
}

/* Bit beliefs L_v = pi_v + sum over c in N(v) of m_{c->v} (Preliminaries),
 * added in ascending c, clamped. */
static void beliefs(const tanner* T, const orc_params* P, const float* pi_v, const float* mcv,
                    float* L) {
  for (int32_t v = 0; v < T->n; ++v) {
    float acc = pi_v[v];
    for (int32_t i = T->vptr[v]; i < T->vptr[v + 1]; ++i) acc = acc + mcv[T->vedge[i]];
    L[v] = clampf_(acc, P->clamp);
  }
}

/* One BP sweep (check phase, then qubit phase) on caller-owned arrays, for
 * the gauge-covariance pin. pi_v has n entries. */
int32_t orc_bp_sweep(int32_t m, int32_t n, const int32_t* rowptr, const int32_t* col,
                     const orc_params* P, const float* pi_v, const uint8_t* s, const float* mvc_in,
                     float* mcv_out, float* mvc_out) {
  tanner T;
  if (tanner_init(&T, m, n, rowptr, col)) return -2;
  check_phase(&T, P, mvc_in, s, mcv_out);
  var_phase(&T, P, pi_v, mcv_out, mvc_out);
  tanner_free(&T);
  return 0;
}

/* Combination of one round's move requests into the flip vector f (n
 * entries, cleared here). Request i is check req_c[i] asking to flip qubit
 * req_v[i] at ring time req_key[i]; every check makes at most one request,
 * and s is the syndrome at the start of the move step. */
typedef struct { uint32_t key; int32_t c, v; } orc_request;

static int cmp_request(const void* a, const void* b) {
  const orc_request* x = (const orc_request*)a;
  const orc_request* y = (const orc_request*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return (x->c > y->c) - (x->c < y->c);
}

static int32_t resolve_moves(const tanner* T, int32_t conflict, const uint8_t* s, int32_t nreq,
                             orc_request* req, uint8_t* f) {
  memset(f, 0, (size_t)T->n);
  if (conflict == ORC_CONFLICT_OR) {
    for (int32_t i = 0; i < nreq; ++i) f[req[i].v] = 1;
  } else if (conflict == ORC_CONFLICT_XOR) {
    for (int32_t i = 0; i < nreq; ++i) f[req[i].v] ^= 1;
  } else if (conflict == ORC_CONFLICT_SEQUENTIAL) {
    qsort(req, (size_t)nreq, sizeof(orc_request), cmp_request);
    /* a check's requests (one per qubit of a multi-qubit move) are adjacent
     * after the sort and apply together: all of them if the check is active
     * before the first, none otherwise */
    uint8_t x = 0;
    for (int32_t i = 0; i < nreq; ++i) {
      if (i == 0 || req[i].c != req[i - 1].c || req[i].key != req[i - 1].key) {
        /* the check's syndrome now: s_c plus the moves applied so far */
        x = s[req[i].c];
        for (int32_t k = T->rowptr[req[i].c]; k < T->rowptr[req[i].c + 1]; ++k) x ^= f[T->col[k]];
      }
      if (x & 1) f[req[i].v] ^= 1;
    }
  } else {
    return -1;
  }
  return 0;
}

/* The combination rule on its own, for the pins: requests given as arrays,
 * f [n] out. Returns 0, -1 for an unknown rule, -2 when out of memory. */
int32_t orc_resolve_moves(int32_t m, int32_t n, const int32_t* rowptr, const int32_t* col,
                          int32_t conflict, const uint8_t* s, int32_t nreq, const int32_t* req_c,
                          const int32_t* req_v, const uint32_t* req_key, uint8_t* f) {
  tanner T;
  if (tanner_init(&T, m, n, rowptr, col)) return -2;
  orc_request* req = (orc_request*)malloc(sizeof(orc_request) * (size_t)(nreq > 0 ? nreq : 1));
  if (!req) {
    tanner_free(&T);
    return -2;
  }
  for (int32_t i = 0; i < nreq; ++i) {
    req[i].key = req_key[i];
    req[i].c = req_c[i];
    req[i].v = req_v[i];
  }
  int32_t rc = resolve_moves(&T, conflict, s, nreq, req, f);
  free(req);
  tanner_free(&T);
  return rc;
}

/* ------------------------------------------------------------------------
 * The round-discretised check-centric machine (Algorithm 1).
 *
 * Per shot: z = 0, s = H e0, all messages +0 (the algorithm's m(0) = 0).
 * Each round r = 0, 1, ...:
 *   1. `iters` BP sweeps on the current syndrome (messages are never reset);
 *   2. beliefs L_v;
 *   3. every check whose clock rang (word 0 of
 *      Philox(seed, (shot_lo, shot_hi, c, 16 r + 1)) below
 *      floor(mask_density 2^32)) and which is active (s_c = 1) computes
 *      Evidence: Lmax = max over v in N(c) of L_v; Pr(e_v = 1 | s) >= 1/d_c
 *      is sigma(L) >= 1/d_c, i.e. L >= -log(d_c - 1). If it holds, the check
 *      picks its LocalMove: the qubits with L_v == Lmax (in ascending order)
 *      are the ties, and word 1 of the same Philox output picks tie number
 *      floor(w1 * ntie / 2^32). The requests combine by the conflict rule
 *      (OR by default: a qubit chosen by several checks flips once);
 *   4. z ^= f; s = H (e0 ^ z), which equals s ^ H f (the syndrome update);
 *   5. if s = 0 for the first time, t_clr = r + 1.
 * t_clr = 0 if H e0 = 0 and -1 if the syndrome never clears.
 *
 * Outputs per shot: z [n], s [m], t_clr, and optionally the beliefs of the
 * final message state L [n]. For a single shot the per-round syndromes and
 * corrections can be traced (s_trace [rounds][m], z_trace [rounds][n]).
 * Returns 0, or -3 if the internal syndrome-update identity check fails.
 * ---------------------------------------------------------------------- */
/* The machine from a given start syndrome s0 (s0 = H e0 for a decode of
 * e0), its rounds numbered r0, r0 + 1, ... for the clock words. */
static int32_t decode_core(const tanner* T, const orc_params* P, const float* thr,
                           uint64_t R_bound, float pi, const uint8_t* s0, uint64_t shot, int32_t r0,
                           uint8_t* z, uint8_t* s, int32_t* tclr, float* L_out, uint8_t* s_trace,
                           uint8_t* z_trace) {
  const int32_t m = T->m, n = T->n, E = T->E;
  float* mvc = (float*)calloc((size_t)(E > 0 ? E : 1), sizeof(float));
  float* mcv = (float*)calloc((size_t)(E > 0 ? E : 1), sizeof(float));
  float* L = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
  float* piv = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
  uint8_t* f = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  uint8_t* r_err = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  uint8_t* s_new = (uint8_t*)malloc((size_t)(m > 0 ? m : 1));
  /* at most one request per edge (a multi-qubit move requests each qubit) */
  orc_request* req = (orc_request*)malloc(sizeof(orc_request) * (size_t)(E > m ? E : (m > 0 ? m : 1)));
  int32_t rc = 0;
  if (!mvc || !mcv || !L || !piv || !f || !r_err || !s_new || !req) {
    rc = -2;
    goto done;
  }
  for (int32_t v = 0; v < n; ++v) { piv[v] = pi; z[v] = 0; }
  int any = 0;
  for (int32_t c = 0; c < m; ++c) {
    s[c] = s0[c] & 1u;
    any |= s[c];
  }
  *tclr = any ? -1 : 0;

  for (int32_t rr = 0; rr < P->rounds; ++rr) {
    const int32_t r = r0 + rr;
    if (P->retire && *tclr >= 0) break;
    for (int32_t it = 0; it < P->iters; ++it) {
      check_phase(T, P, mvc, s, mcv);
      var_phase(T, P, piv, mcv, mvc);
    }
    beliefs(T, P, piv, mcv, L);
    int32_t nreq = 0;
    for (int32_t c = 0; c < m; ++c) {
      if (!s[c]) continue;
      uint32_t w[4];
      philox_for(P->seed, shot, (uint32_t)c, ((uint32_t)r << 4) | 1u, w);
      if (!((uint64_t)w[0] < R_bound)) continue;
      int32_t b = T->rowptr[c], dc = T->rowptr[c + 1] - b;
      if (dc == 0) continue;
      float Lmax = L[T->col[b]];
      for (int32_t j = 1; j < dc; ++j)
        if (L[T->col[b + j]] > Lmax) Lmax = L[T->col[b + j]];
      if (P->evidence && !(Lmax >= thr[dc])) continue;
      if (P->move == ORC_MOVE_MULTI) {
        /* every qubit of N(c) with L_v > 0, else the LocalMove qubit */
        int32_t npos = 0;
        for (int32_t j = 0; j < dc; ++j) {
          if (L[T->col[b + j]] > 0.0f) {
            req[nreq].key = w[2];
            req[nreq].c = c;
            req[nreq].v = T->col[b + j];
            nreq++;
            npos++;
          }
        }
        if (npos > 0) continue;
      }
      uint32_t ntie = 0;
      for (int32_t j = 0; j < dc; ++j) ntie += (L[T->col[b + j]] == Lmax) ? 1u : 0u;
      uint32_t pick = (uint32_t)(((uint64_t)w[1] * (uint64_t)ntie) >> 32);
      for (int32_t j = 0; j < dc; ++j) {
        if (L[T->col[b + j]] == Lmax) {
          if (pick == 0) {
            req[nreq].key = w[2];
            req[nreq].c = c;
            req[nreq].v = T->col[b + j];
            nreq++;
            break;
          }
          pick--;
        }
      }
    }
    if (resolve_moves(T, P->conflict, s, nreq, req, f)) {
      rc = -1;
      goto done;
    }
    for (int32_t v = 0; v < n; ++v) z[v] ^= f[v];
    if (P->gauge) {
      for (int32_t v = 0; v < n; ++v) {
        if (!f[v]) continue;
        piv[v] = -piv[v];
        for (int32_t i = T->vptr[v]; i < T->vptr[v + 1]; ++i) {
          int32_t e = T->vedge[i];
          mcv[e] = -mcv[e];
          mvc[e] = -mvc[e];
        }
      }
    }
    /* re-measure, s = s0 ^ H z (= H (e0 ^ z)), and check it against the
     * incremental update s ^ H f */
    orc_syndrome(m, n, T->rowptr, T->col, z, 1, s_new);
    any = 0;
    for (int32_t c = 0; c < m; ++c) {
      s_new[c] ^= s0[c] & 1u;
      uint8_t x = s[c];
      for (int32_t k = T->rowptr[c]; k < T->rowptr[c + 1]; ++k) x ^= f[T->col[k]];
      if (x != s_new[c]) rc = -3;
      s[c] = s_new[c];
      any |= s[c];
    }
    if (!any && *tclr < 0) *tclr = rr + 1;
    if (s_trace) memcpy(s_trace + (size_t)rr * m, s, (size_t)m);
    if (z_trace) memcpy(z_trace + (size_t)rr * n, z, (size_t)n);
  }
  if (L_out) beliefs(T, P, piv, mcv, L_out);
done:
  free(mvc); free(mcv); free(L); free(piv); free(f); free(r_err); free(s_new); free(req);
  return rc;
}

/* The machine on the initial error e0 (rounds numbered from 0). */
static int32_t decode_one(const tanner* T, const orc_params* P, const float* thr,
                          uint64_t R_bound, float pi, const uint8_t* e0, uint64_t shot,
                          uint8_t* z, uint8_t* s, int32_t* tclr, float* L_out, uint8_t* s_trace,
                          uint8_t* z_trace) {
  uint8_t* s0 = (uint8_t*)malloc((size_t)(T->m > 0 ? T->m : 1));
  if (!s0) return -2;
  orc_syndrome(T->m, T->n, T->rowptr, T->col, e0, 1, s0);
  int32_t rc = decode_core(T, P, thr, R_bound, pi, s0, shot, 0, z, s, tclr, L_out, s_trace, z_trace);
  free(s0);
  return rc;
}

/* The machine from given start syndromes (s0 [nshots][m]), rounds numbered
 * from r0: the building block of the online decoder, exposed for its pins. */
int32_t orc_decode_syndrome(int32_t m, int32_t n, const int32_t* rowptr, const int32_t* col,
                            const orc_params* P, const uint8_t* s0, uint64_t shot0, int32_t r0,
                            int32_t nshots, uint8_t* z_out, uint8_t* s_out, int32_t* tclr_out);

/* thr[d] = -log(d - 1) rounded to float, the Evidence bound for degree d
 * (thr[1] = +inf: a degree-1 check never has evidence; thr[2] = -0). */
void orc_evidence_thresholds(int32_t dmax, float* thr) {
  for (int32_t d = 0; d <= dmax; ++d) thr[d] = (d <= 1) ? INFINITY : (float)(-log((double)(d - 1)));
}

int32_t orc_decode(int32_t m, int32_t n, const int32_t* rowptr, const int32_t* col,
                   const orc_params* P, const uint8_t* e0, uint64_t shot0, int32_t nshots,
                   uint8_t* z_out, uint8_t* s_out, int32_t* tclr_out, float* L_out,
                   uint8_t* s_trace, uint8_t* z_trace, int32_t nthreads) {
  tanner T;
  if (tanner_init(&T, m, n, rowptr, col)) return -2;
  int32_t dmax = 0;
  for (int32_t c = 0; c < m; ++c)
    if (rowptr[c + 1] - rowptr[c] > dmax) dmax = rowptr[c + 1] - rowptr[c];
  float* thr = (float*)malloc(sizeof(float) * (size_t)(dmax + 1));
  orc_evidence_thresholds(dmax, thr);
  const float pi = (float)log(P->q / (1.0 - P->q));
  const uint64_t R_bound = orc_bernoulli_bound(P->mask_density);
  int32_t rc = 0;
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads) reduction(min : rc)
  for (int32_t i = 0; i < nshots; ++i) {
    int32_t r1 = decode_one(&T, P, thr, R_bound, pi, e0 + (size_t)i * n, shot0 + (uint64_t)i,
                            z_out + (size_t)i * n, s_out + (size_t)i * m, tclr_out + i,
                            L_out ? L_out + (size_t)i * n : NULL,
                            (nshots == 1) ? s_trace : NULL, (nshots == 1) ? z_trace : NULL);
    if (r1 < rc) rc = r1;
  }
  free(thr);
  tanner_free(&T);
  return rc;
}

/* ------------------------------------------------------------------------
 * The continuous-time machine (Algorithm 1 as stated; SM "Numerical
 * details" for its simulation): BP relaxes by tau dm/dt = F_BP(m; S) - m,
 * integrated with Euler steps of dt, while unit-rate Poisson clocks ring at
 * the checks. Only active checks can act, so the next ring is simulated by
 * a waiting time ~ Exp(|S|) and a uniformly chosen active check.
 *
 * One Euler step (the Jacobi form: both message directions from the state
 * before the step), lambda = (float)(dt / tau):
 *   Fc(c,v) = check rule of the current m_{v->c} and s   (BP-LLR2),
 *   Fv(v,c) = clamp(pi + sum over c' in N(v)\c of m_{c'->v}) (BP-LLR1),
 *   m_{c->v} <- clamp(m_{c->v} + lambda (Fc - m_{c->v})),
 *   m_{v->c} <- clamp(m_{v->c} + lambda (Fv - m_{v->c})).
 *
 * Events. Event j draws Philox(key = seed, ctr = (shot_lo, shot_hi, j, 2))
 * = (w0, w1, w2, w3): its waiting time is -ln((w0 + 1) 2^-32) / |S| (FP64,
 * with |S| the number of active checks after event j - 1), the ringing
 * check is active check number floor(w1 |S| / 2^32) in ascending order, and
 * w2 breaks LocalMove ties as in the round machine. An event at time T acts
 * on the BP state after floor-many steps: at step k (time k dt) every event
 * with T <= k dt is applied, in order, before the next Euler step. A ringing
 * check with Evidence (Lmax >= -log(d_c - 1) over the beliefs of N(c))
 * flips its LocalMove qubit: z_v ^= 1, s ^= H e_v.
 *
 * t_clr is the time of the event that clears the syndrome (0 if H e0 = 0).
 * The run stops unsuccessfully after K = max_steps Euler steps (events up
 * to time K dt are applied); then t_clr = -1.
 * ---------------------------------------------------------------------- */

/* ln(u) for 0 < u <= 1 in double: u = f 2^e with f in [sqrt(1/2), sqrt(2)),
 * ln f = 2 atanh(s) = 2 s (1 + s^2/3 + s^4/5 + ... + s^24/25) with
 * s = (f - 1) / (f + 1), |s| <= 0.1716, ln u = e ln2 + ln f. */
double orc_ln_unit(double u) {
  uint64_t b;
  memcpy(&b, &u, 8);
  int32_t e = (int32_t)((b >> 52) & 0x7ffu) - 1023;
  uint64_t fb = (b & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
  double f;
  memcpy(&f, &fb, 8);
  if (f > 1.4142135623730951) {
    f = f * 0.5;
    e = e + 1;
  }
  double s = (f - 1.0) / (f + 1.0);
  double s2 = s * s;
  double p = 1.0 / 25.0;
  for (int32_t k = 11; k >= 0; --k) p = p * s2 + 1.0 / (double)(2 * k + 1);
  return (double)e * 0.6931471805599453 + 2.0 * s * p;
}

typedef struct {
  int32_t bp;
  float alpha;
  double q;
  float clamp;
  double dt;
  double tau;
  int32_t max_steps;  /* Euler steps before an unsuccessful stop */
  int32_t evidence;
  uint64_t seed;
} orc_ctm_params;

/* waiting time of event j at rate nS */
static double ctm_wait(uint64_t seed, uint64_t shot, uint32_t j, int32_t nS, uint32_t w[4]) {
  philox_for(seed, shot, j, 2u, w);
  double u = ((double)w[0] + 1.0) * (1.0 / 4294967296.0);
  return -orc_ln_unit(u) / (double)nS;
}

/* One Euler step of the damped Jacobi BP on caller arrays. */
static void ctm_euler(const tanner* T, const orc_params* P, float pi, float lam, const uint8_t* s,
                      float* mcv, float* mvc, float* Fc, float* Fv) {
  for (int32_t c = 0; c < T->m; ++c) {
    int32_t b = T->rowptr[c], dc = T->rowptr[c + 1] - b;
    for (int32_t j = 0; j < dc; ++j) Fc[b + j] = check_rule(P, mvc + b, dc, j, s[c]);
  }
  for (int32_t v = 0; v < T->n; ++v) {
    int32_t b = T->vptr[v], dv = T->vptr[v + 1] - b;
    for (int32_t j = 0; j < dv; ++j) {
      float acc = pi;
      for (int32_t i = 0; i < dv; ++i)
        if (i != j) acc = acc + mcv[T->vedge[b + i]];
      Fv[T->vedge[b + j]] = clampf_(acc, P->clamp);
    }
  }
  for (int32_t e = 0; e < T->E; ++e) {
    mcv[e] = clampf_(mcv[e] + lam * (Fc[e] - mcv[e]), P->clamp);
    mvc[e] = clampf_(mvc[e] + lam * (Fv[e] - mvc[e]), P->clamp);
  }
}

static void ctm_set(const orc_ctm_params* C, orc_params* P) {
  memset(P, 0, sizeof(*P));
  P->bp = C->bp;
  P->alpha = C->alpha;
  P->q = C->q;
  P->clamp = C->clamp;
  P->evidence = C->evidence;
  P->seed = C->seed;
}

/* K Euler steps from m = 0 on a fixed syndrome s (for pins); final m_{c->v}
 * and m_{v->c} in edge order. */
int32_t orc_ctm_bp_steps(int32_t m, int32_t n, const int32_t* rowptr, const int32_t* col,
                         const orc_ctm_params* C, const uint8_t* s, int32_t K, float* mcv_out,
                         float* mvc_out) {
  tanner T;
  if (tanner_init(&T, m, n, rowptr, col)) return -2;
  orc_params P;
  ctm_set(C, &P);
  const float pi = (float)log(C->q / (1.0 - C->q));
  const float lam = (float)(C->dt / C->tau);
  size_t E = (size_t)(T.E > 0 ? T.E : 1);
  float* Fc = (float*)malloc(sizeof(float) * E);
  float* Fv = (float*)malloc(sizeof(float) * E);
  for (int32_t e = 0; e < T.E; ++e) mcv_out[e] = mvc_out[e] = 0.0f;
  for (int32_t k = 0; k < K; ++k) ctm_euler(&T, &P, pi, lam, s, mcv_out, mvc_out, Fc, Fv);
  free(Fc);
  free(Fv);
  tanner_free(&T);
  return 0;
}

/* Per shot. trace (one shot only, may be NULL): per event j, 4 doubles:
 * time, |S| before it, the ringing check, the flipped qubit (-1 if none). */
static int32_t ctm_one(const tanner* T, const orc_ctm_params* C, const orc_params* P,
                       const float* thr, float pi, float lam, const uint8_t* e0, uint64_t shot,
                       uint8_t* z, uint8_t* s, double* tclr, int32_t* counts, double* trace,
                       int32_t trace_cap) {
  const int32_t m = T->m, n = T->n;
  const size_t E = (size_t)(T->E > 0 ? T->E : 1);
  float* mcv = (float*)calloc(E, sizeof(float));
  float* mvc = (float*)calloc(E, sizeof(float));
  float* Fc = (float*)malloc(sizeof(float) * E);
  float* Fv = (float*)malloc(sizeof(float) * E);
  float Lv[64];
  if (!mcv || !mvc || !Fc || !Fv) {
    free(mcv); free(mvc); free(Fc); free(Fv);
    return -2;
  }
  for (int32_t v = 0; v < n; ++v) z[v] = 0;
  orc_syndrome(m, n, T->rowptr, T->col, e0, 1, s);
  int32_t nS = 0;
  for (int32_t c = 0; c < m; ++c) nS += s[c];
  int32_t events = 0, moves = 0;
  uint32_t j = 0;
  *tclr = (nS == 0) ? 0.0 : -1.0;
  double Tev = 0.0;
  uint32_t w[4];
  if (nS > 0) Tev = ctm_wait(C->seed, shot, j, nS, w);
  for (int32_t k = 0; nS > 0; ++k) {
    const double tk = (double)k * C->dt;
    while (nS > 0 && Tev <= tk) {
      philox_for(C->seed, shot, j, 2u, w);
      uint32_t idx = (uint32_t)(((uint64_t)w[1] * (uint64_t)nS) >> 32);
      int32_t c = 0;
      for (; c < m; ++c)
        if (s[c]) {
          if (idx == 0) break;
          idx--;
        }
      int32_t b = T->rowptr[c], dc = T->rowptr[c + 1] - b;
      int32_t flipped = -1;
      if (dc > 0 && dc <= 64) {
        float Lmax = 0.0f;
        for (int32_t jj = 0; jj < dc; ++jj) {
          int32_t v = T->col[b + jj];
          float acc = pi;
          for (int32_t i = T->vptr[v]; i < T->vptr[v + 1]; ++i) acc = acc + mcv[T->vedge[i]];
          Lv[jj] = clampf_(acc, C->clamp);
          if (jj == 0 || Lv[jj] > Lmax) Lmax = Lv[jj];
        }
        if (!C->evidence || Lmax >= thr[dc]) {
          uint32_t ntie = 0;
          for (int32_t jj = 0; jj < dc; ++jj) ntie += (Lv[jj] == Lmax) ? 1u : 0u;
          uint32_t pick = (uint32_t)(((uint64_t)w[2] * (uint64_t)ntie) >> 32);
          for (int32_t jj = 0; jj < dc; ++jj)
            if (Lv[jj] == Lmax) {
              if (pick == 0) {
                flipped = T->col[b + jj];
                break;
              }
              pick--;
            }
        }
      }
      if (trace && events < trace_cap) {
        trace[4 * events + 0] = Tev;
        trace[4 * events + 1] = (double)nS;
        trace[4 * events + 2] = (double)c;
        trace[4 * events + 3] = (double)flipped;
      }
      if (flipped >= 0) {
        z[flipped] ^= 1u;
        for (int32_t i = T->vptr[flipped]; i < T->vptr[flipped + 1]; ++i) {
          int32_t c2 = 0;
          /* the check of edge vedge[i] */
          int32_t e = T->vedge[i];
          while (T->rowptr[c2 + 1] <= e) c2++;
          s[c2] ^= 1u;
          nS += s[c2] ? 1 : -1;
        }
        moves++;
      }
      events++;
      j++;
      if (nS == 0) {
        *tclr = Tev;
        break;
      }
      Tev = Tev + ctm_wait(C->seed, shot, j, nS, w);
    }
    if (nS == 0 || k >= C->max_steps) break;
    ctm_euler(T, P, pi, lam, s, mcv, mvc, Fc, Fv);
  }
  counts[0] = events;
  counts[1] = moves;
  free(mcv); free(mvc); free(Fc); free(Fv);
  return 0;
}

int32_t orc_ctm_decode(int32_t m, int32_t n, const int32_t* rowptr, const int32_t* col,
                       const orc_ctm_params* C, const uint8_t* e0, uint64_t shot0, int32_t nshots,
                       uint8_t* z_out, uint8_t* s_out, double* tclr_out, int32_t* counts_out,
                       double* trace, int32_t trace_cap, int32_t nthreads) {
  tanner T;
  if (tanner_init(&T, m, n, rowptr, col)) return -2;
  int32_t dmax = 0;
  for (int32_t c = 0; c < m; ++c)
    if (rowptr[c + 1] - rowptr[c] > dmax) dmax = rowptr[c + 1] - rowptr[c];
  float* thr = (float*)malloc(sizeof(float) * (size_t)(dmax + 1));
  orc_evidence_thresholds(dmax, thr);
  orc_params P;
  ctm_set(C, &P);
  const float pi = (float)log(C->q / (1.0 - C->q));
  const float lam = (float)(C->dt / C->tau);
  int32_t rc = 0;
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(min : rc)
  for (int32_t i = 0; i < nshots; ++i) {
    int32_t r1 = ctm_one(&T, C, &P, thr, pi, lam, e0 + (size_t)i * n, shot0 + (uint64_t)i,
                         z_out + (size_t)i * n, s_out + (size_t)i * m, tclr_out + i,
                         counts_out + 2 * (size_t)i, (nshots == 1) ? trace : NULL, trace_cap);
    if (r1 < rc) rc = r1;
  }
  free(thr);
  tanner_free(&T);
  return rc;
}

void orc_vec_ln_unit(const double* x, int32_t k, double* y) {
  for (int32_t i = 0; i < k; ++i) y[i] = orc_ln_unit(x[i]);
}

/* ------------------------------------------------------------------------
 * GF(2) linear algebra on bit-packed rows, for the success test.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t rows, words;
  uint64_t* a;    /* rows x words */
  int32_t* pivot; /* pivot column of each reduced row */
  int32_t rank;
} gf2_basis;

static void pack_rows(int32_t rows, int32_t n, const int32_t* rowptr, const int32_t* col,
                      int32_t words, uint64_t* a) {
  memset(a, 0, sizeof(uint64_t) * (size_t)rows * words);
  for (int32_t r = 0; r < rows; ++r)
    for (int32_t k = rowptr[r]; k < rowptr[r + 1]; ++k)
      a[(size_t)r * words + (col[k] >> 6)] ^= (uint64_t)1 << (col[k] & 63);
  (void)n;
}

/* Row-reduce by Gaussian elimination; the reduced rows span the row space. */
static int gf2_basis_init(gf2_basis* B, int32_t rows, int32_t n, const int32_t* rowptr,
                          const int32_t* col) {
  B->rows = rows;
  B->words = (n + 63) / 64;
  B->a = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(rows > 0 ? rows : 1) * B->words);
  B->pivot = (int32_t*)malloc(sizeof(int32_t) * (size_t)(rows > 0 ? rows : 1));
  if (!B->a || !B->pivot) return -2;
  pack_rows(rows, n, rowptr, col, B->words, B->a);
  int32_t rank = 0;
  for (int32_t c = 0; c < n && rank < rows; ++c) {
    int32_t w = c >> 6;
    uint64_t bit = (uint64_t)1 << (c & 63);
    int32_t piv = -1;
    for (int32_t r = rank; r < rows; ++r)
      if (B->a[(size_t)r * B->words + w] & bit) { piv = r; break; }
    if (piv < 0) continue;
    if (piv != rank)
      for (int32_t k = 0; k < B->words; ++k) {
        uint64_t t = B->a[(size_t)piv * B->words + k];
        B->a[(size_t)piv * B->words + k] = B->a[(size_t)rank * B->words + k];
        B->a[(size_t)rank * B->words + k] = t;
      }
    for (int32_t r = 0; r < rows; ++r)
      if (r != rank && (B->a[(size_t)r * B->words + w] & bit))
        for (int32_t k = 0; k < B->words; ++k)
          B->a[(size_t)r * B->words + k] ^= B->a[(size_t)rank * B->words + k];
    B->pivot[rank] = c;
    rank++;
  }
  B->rank = rank;
  return 0;
}

static void gf2_basis_free(gf2_basis* B) { free(B->a); free(B->pivot); }

int32_t orc_gf2_rank(int32_t rows, int32_t n, const int32_t* rowptr, const int32_t* col) {
  gf2_basis B;
  if (gf2_basis_init(&B, rows, n, rowptr, col)) return -2;
  int32_t r = B.rank;
  gf2_basis_free(&B);
  return r;
}

/* Is the 0/1 vector x (length n) in the row space of the basis?
 * Equivalent to rank([G; x]) == rank(G). */
static int in_row_space(const gf2_basis* B, int32_t n, const uint8_t* x, uint64_t* work) {
  memset(work, 0, sizeof(uint64_t) * (size_t)B->words);
  for (int32_t v = 0; v < n; ++v)
    if (x[v] & 1u) work[v >> 6] ^= (uint64_t)1 << (v & 63);
  for (int32_t r = 0; r < B->rank; ++r) {
    int32_t c = B->pivot[r];
    if (work[c >> 6] & ((uint64_t)1 << (c & 63)))
      for (int32_t k = 0; k < B->words; ++k) work[k] ^= B->a[(size_t)r * B->words + k];
  }
  for (int32_t k = 0; k < B->words; ++k)
    if (work[k]) return 0;
  return 1;
}

/* Decoder failure (Preliminaries): fail unless (1) H (e0 ^ z) = 0 and (2)
 * e0 ^ z lies in row(G). */
int32_t orc_logical_failure(int32_t m, int32_t n, const int32_t* h_rowptr, const int32_t* h_col,
                            int32_t mg, const int32_t* g_rowptr, const int32_t* g_col,
                            const uint8_t* e0, const uint8_t* z, int32_t nshots, uint8_t* fail_out) {
  gf2_basis B;
  if (gf2_basis_init(&B, mg, n, g_rowptr, g_col)) return -2;
  uint8_t* r = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  uint8_t* s = (uint8_t*)malloc((size_t)(m > 0 ? m : 1));
  uint64_t* work = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(B.words > 0 ? B.words : 1));
  for (int32_t i = 0; i < nshots; ++i) {
    for (int32_t v = 0; v < n; ++v) r[v] = (uint8_t)((e0[(size_t)i * n + v] ^ z[(size_t)i * n + v]) & 1u);
    orc_syndrome(m, n, h_rowptr, h_col, r, 1, s);
    int any = 0;
    for (int32_t c = 0; c < m; ++c) any |= s[c];
    fail_out[i] = (uint8_t)(any || !in_row_space(&B, n, r, work));
  }
  free(r); free(s); free(work);
  gf2_basis_free(&B);
  return 0;
}

/* ------------------------------------------------------------------------
 * Online decoding in overlapping spacetime windows (Discussion: new faults
 * and syndrome information keep arriving; the Tanner graph is promoted to a
 * spacetime decoding graph and the local dynamics runs inside overlapping
 * spacetime windows). The paper fixes neither the noise model nor the window
 * rule; the reading:
 *   noise      N syndrome rounds t = 1..N. Before round t every qubit gets a
 *              new Z error e_t[v] ~ Bernoulli(p); round t measures
 *              m_t = H E_t ^ eps_t with E_t = e_1 ^ ... ^ e_t and
 *              measurement errors eps_t[c] ~ Bernoulli(p_meas), except that
 *              the last round is perfect (eps_N = 0). Words: e_t[v] is word
 *              (v mod 4) of Philox(seed, (shot_lo, shot_hi, floor(v/4),
 *              16 t + 3)), eps_t[c] word (c mod 4) of Philox(seed, (shot_lo,
 *              shot_hi, floor(c/4), 16 t + 4)), each below floor(rate 2^32).
 *   detectors  D_t = m_t ^ m_{t-1} (m_0 = 0) = H e_t ^ eps_t ^ eps_{t-1}.
 *   graph      one variable per e_t[v] and per eps_t[c] (t < N), one check
 *              per detector (t, c) holding e_t[v] for v in N(c), eps_{t-1}[c]
 *              and eps_t[c] where they exist; one prior q for all variables.
 *   windows    window k covers rounds k C + 1 .. min(k C + W, N); the last
 *              window is the first that reaches round N. Its check (tau, c)
 *              (round k C + 1 + tau) gets the syndrome D, with the committed
 *              correction of eps_{kC}[c] added on tau = 0. The round machine
 *              decodes it from fresh messages, its rounds numbered from k R
 *              (R rounds per window), so every window draws its own clock
 *              words. The window's variables of its first C rounds (all of
 *              them in the last window) are committed: their data
 *              corrections add to the running correction z, and the
 *              measurement corrections of the last committed round carry into
 *              the next window.
 *   result     z, and the failure of the offline test applied to the final
 *              error E_N: H (E_N ^ z) != 0 or E_N ^ z not in row(G).
 * Window variables (w rounds, local round tau, measurement variables for the
 * first w_eps rounds: w_eps = w, or w - 1 when the window ends with the
 * perfect round): data (tau, v) is tau n + v, measurement (tau, c) is
 * w n + tau m + c; check (tau, c) is tau m + c.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t rounds_total; /* N syndrome rounds, the last one perfect */
  int32_t window;       /* W rounds per window */
  int32_t commit;       /* C rounds committed per window, 1 <= C <= W */
  double p;             /* data error rate per qubit and round */
  double p_meas;        /* measurement error rate per check and round */
} orc_online_params;

/* Spacetime errors of one shot: e [N][n], eps [N][m] (the last row 0). */
static void online_noise_one(int32_t n, int32_t m, const orc_online_params* O, uint64_t seed,
                             uint64_t shot, uint8_t* e, uint8_t* eps) {
  const uint64_t bd = orc_bernoulli_bound(O->p), bm = orc_bernoulli_bound(O->p_meas);
  const int32_t N = O->rounds_total;
  uint32_t w[4];
  for (int32_t t = 1; t <= N; ++t) {
    for (int32_t v = 0; v < n; ++v) {
      philox_for(seed, shot, (uint32_t)(v >> 2), ((uint32_t)t << 4) | 3u, w);
      e[(size_t)(t - 1) * n + v] = (uint8_t)((uint64_t)w[v & 3] < bd);
    }
    for (int32_t c = 0; c < m; ++c) {
      uint8_t x = 0;
      if (t < N) {
        philox_for(seed, shot, (uint32_t)(c >> 2), ((uint32_t)t << 4) | 4u, w);
        x = (uint8_t)((uint64_t)w[c & 3] < bm);
      }
      eps[(size_t)(t - 1) * m + c] = x;
    }
  }
}

void orc_online_noise(int32_t n, int32_t m, const orc_online_params* O, uint64_t seed,
                      uint64_t shot0, int32_t nshots, uint8_t* e_out, uint8_t* eps_out) {
  const size_t N = (size_t)O->rounds_total;
  for (int32_t i = 0; i < nshots; ++i)
    online_noise_one(n, m, O, seed, shot0 + (uint64_t)i, e_out + (size_t)i * N * n,
                     eps_out + (size_t)i * N * m);
}

/* The CSR of a window of w rounds with measurement variables for its first
 * w_eps rounds. Returns the number of variables, or -2 without memory. */
static int32_t window_csr(const tanner* T, int32_t w, int32_t w_eps, int32_t** rowptr, int32_t** col) {
  const int32_t m = T->m, n = T->n;
  int32_t* rp = (int32_t*)malloc(sizeof(int32_t) * ((size_t)w * m + 1));
  int32_t* cl = (int32_t*)malloc(sizeof(int32_t) * ((size_t)w * (T->E + 2 * m) + 1));
  if (!rp || !cl) {
    free(rp);
    free(cl);
    return -2;
  }
  int32_t k = 0;
  rp[0] = 0;
  for (int32_t tau = 0; tau < w; ++tau) {
    for (int32_t c = 0; c < m; ++c) {
      for (int32_t e = T->rowptr[c]; e < T->rowptr[c + 1]; ++e) cl[k++] = tau * n + T->col[e];
      if (tau >= 1 && tau - 1 < w_eps) cl[k++] = w * n + (tau - 1) * m + c;
      if (tau < w_eps) cl[k++] = w * n + tau * m + c;
      rp[tau * m + c + 1] = k;
    }
  }
  *rowptr = rp;
  *col = cl;
  return w * n + w_eps * m;
}

/* The window layout of a run: nwin windows, window k starting at round
 * k C + 1; the last has w_last rounds. */
static void window_layout(const orc_online_params* O, int32_t* nwin, int32_t* w_last) {
  const int32_t N = O->rounds_total, W = O->window, C = O->commit;
  int32_t k = 0;
  while (k * C + W < N) ++k;
  *nwin = k + 1;
  *w_last = N - k * C;
}

/* Online decode of nshots shots (ids shot0 + i). With e_in / eps_in
 * ([nshots][N][n], [nshots][N][m]; both or neither) the given errors are
 * used instead of sampled ones. Outputs: z [nshots][n], E [nshots][n] (the
 * final error), fail [nshots], cleared [nshots] (windows whose syndrome
 * cleared); with one shot, trace_s [nwin][W m] and trace_z [nwin][W (n + m)]
 * record each window's syndrome and correction (rows zero-padded).
 * Returns 0, -1 for bad parameters, -2 without memory, -3 if a window's
 * syndrome update identity fails. */
int32_t orc_online_decode(int32_t m, int32_t n, const int32_t* rowptr, const int32_t* col, int32_t mg,
                          const int32_t* g_rowptr, const int32_t* g_col, const orc_params* P,
                          const orc_online_params* O, uint64_t shot0, int32_t nshots,
                          const uint8_t* e_in, const uint8_t* eps_in, uint8_t* z_out, uint8_t* E_out,
                          uint8_t* fail_out, int32_t* cleared_out, uint8_t* trace_s, uint8_t* trace_z,
                          int32_t nthreads) {
  const int32_t N = O->rounds_total, W = O->window, C = O->commit;
  if (N < 1 || W < 1 || C < 1 || C > W || P->rounds < 0) return -1;
  tanner T;
  if (tanner_init(&T, m, n, rowptr, col)) return -2;
  int32_t nwin, w_last;
  window_layout(O, &nwin, &w_last);
  /* the two window shapes: full windows (W rounds, every round with its
   * measurement variables) and the last window (ending with the perfect round) */
  int32_t *rp_full = NULL, *cl_full = NULL, *rp_last = NULL, *cl_last = NULL;
  int32_t nv_full = 0, nv_last = window_csr(&T, w_last, w_last - 1, &rp_last, &cl_last);
  if (nwin > 1) nv_full = window_csr(&T, W, W, &rp_full, &cl_full);
  if (nv_last < 0 || nv_full < 0) {
    tanner_free(&T);
    return -2;
  }
  tanner Tf, Tl;
  int init_f = (nwin > 1) ? tanner_init(&Tf, W * m, nv_full, rp_full, cl_full) : 0;
  int init_l = tanner_init(&Tl, w_last * m, nv_last, rp_last, cl_last);
  const int32_t dmax = T.E > 0 ? 32 : 2;
  float* thr = (float*)malloc(sizeof(float) * (size_t)(dmax + 1));
  orc_evidence_thresholds(dmax, thr);
  const float pi = (float)log(P->q / (1.0 - P->q));
  const uint64_t R_bound = orc_bernoulli_bound(P->mask_density);
  int32_t rc = (init_f || init_l || !thr) ? -2 : 0;
  if (nthreads < 1) nthreads = 1;
  if (rc == 0) {
#pragma omp parallel for schedule(static) num_threads(nthreads) reduction(min : rc)
    for (int32_t i = 0; i < nshots; ++i) {
      const uint64_t shot = shot0 + (uint64_t)i;
      const int32_t nvm = W * (n + m) > n ? W * (n + m) : n;
      uint8_t* e = (uint8_t*)malloc((size_t)N * n);
      uint8_t* eps = (uint8_t*)malloc((size_t)N * m);
      uint8_t* D = (uint8_t*)malloc((size_t)N * m);
      uint8_t* sw = (uint8_t*)malloc((size_t)W * m);
      uint8_t* sout = (uint8_t*)malloc((size_t)W * m);
      uint8_t* zw = (uint8_t*)malloc((size_t)nvm);
      uint8_t* bnd = (uint8_t*)calloc((size_t)m, 1);
      uint8_t* z = z_out + (size_t)i * n;
      uint8_t* E = E_out + (size_t)i * n;
      int32_t r1 = 0;
      if (!e || !eps || !D || !sw || !sout || !zw || !bnd) r1 = -2;
      if (r1 == 0) {
        if (e_in) {
          memcpy(e, e_in + (size_t)i * N * n, (size_t)N * n);
          memcpy(eps, eps_in + (size_t)i * N * m, (size_t)N * m);
          for (int32_t c = 0; c < m; ++c) eps[(size_t)(N - 1) * m + c] = 0; /* perfect last round */
        } else {
          online_noise_one(n, m, O, P->seed, shot, e, eps);
        }
        /* detectors D_t = H e_t ^ eps_t ^ eps_{t-1}; final error E_N */
        for (int32_t t = 0; t < N; ++t) {
          orc_syndrome(m, n, rowptr, col, e + (size_t)t * n, 1, D + (size_t)t * m);
          for (int32_t c = 0; c < m; ++c) {
            D[(size_t)t * m + c] ^= eps[(size_t)t * m + c];
            if (t > 0) D[(size_t)t * m + c] ^= eps[(size_t)(t - 1) * m + c];
          }
        }
        for (int32_t v = 0; v < n; ++v) {
          uint8_t x = 0;
          for (int32_t t = 0; t < N; ++t) x ^= e[(size_t)t * n + v];
          E[v] = x & 1u;
          z[v] = 0;
        }
        int32_t cleared = 0;
        for (int32_t k = 0; k < nwin && r1 == 0; ++k) {
          const int last = (k == nwin - 1);
          const int32_t a = k * C; /* first round of the window, 0-based */
          const int32_t w = last ? w_last : W;
          const tanner* Tw = last ? &Tl : &Tf;
          for (int32_t tau = 0; tau < w; ++tau)
            for (int32_t c = 0; c < m; ++c)
              sw[tau * m + c] = (uint8_t)(D[(size_t)(a + tau) * m + c] ^ (tau == 0 ? bnd[c] : 0));
          int32_t tclr;
          r1 = decode_core(Tw, P, thr, R_bound, pi, sw, shot, k * P->rounds, zw, sout, &tclr, NULL,
                           NULL, NULL);
          cleared += (tclr >= 0);
          const int32_t cr = last ? w : C; /* rounds committed */
          for (int32_t tau = 0; tau < cr; ++tau)
            for (int32_t v = 0; v < n; ++v) z[v] ^= zw[tau * n + v];
          if (!last)
            for (int32_t c = 0; c < m; ++c) bnd[c] = zw[w * n + (cr - 1) * m + c];
          if (trace_s && nshots == 1) {
            memset(trace_s + (size_t)k * W * m, 0, (size_t)W * m);
            memcpy(trace_s + (size_t)k * W * m, sw, (size_t)w * m);
            memset(trace_z + (size_t)k * W * (n + m), 0, (size_t)W * (n + m));
            memcpy(trace_z + (size_t)k * W * (n + m), zw, (size_t)Tw->n);
          }
        }
        if (cleared_out) cleared_out[i] = cleared;
      }
      free(e); free(eps); free(D); free(sw); free(sout); free(zw); free(bnd);
      if (r1 < rc) rc = r1;
    }
  }
  if (rc == 0) rc = orc_logical_failure(m, n, rowptr, col, mg, g_rowptr, g_col, E_out, z_out, nshots, fail_out);
  free(thr);
  if (nwin > 1) tanner_free(&Tf);
  tanner_free(&Tl);
  tanner_free(&T);
  free(rp_full); free(cl_full); free(rp_last); free(cl_last);
  return rc;
}

int32_t orc_decode_syndrome(int32_t m, int32_t n, const int32_t* rowptr, const int32_t* col,
                            const orc_params* P, const uint8_t* s0, uint64_t shot0, int32_t r0,
                            int32_t nshots, uint8_t* z_out, uint8_t* s_out, int32_t* tclr_out) {
  tanner T;
  if (tanner_init(&T, m, n, rowptr, col)) return -2;
  float thr[33];
  orc_evidence_thresholds(32, thr);
  const float pi = (float)log(P->q / (1.0 - P->q));
  const uint64_t R_bound = orc_bernoulli_bound(P->mask_density);
  int32_t rc = 0;
  for (int32_t i = 0; i < nshots && rc == 0; ++i)
    rc = decode_core(&T, P, thr, R_bound, pi, s0 + (size_t)i * m, shot0 + (uint64_t)i, r0,
                     z_out + (size_t)i * n, s_out + (size_t)i * m, tclr_out + i, NULL, NULL, NULL);
  tanner_free(&T);
  return rc;
}

/* The CSR of a window code, for the pins: w rounds, measurement variables
 * for the first w_eps. rowptr_out [w m + 1], col_out [w (E + 2 m)]; returns
 * the number of variables. */
int32_t orc_window_code(int32_t m, int32_t n, const int32_t* rowptr, const int32_t* col, int32_t w,
                        int32_t w_eps, int32_t* rowptr_out, int32_t* col_out) {
  tanner T;
  if (tanner_init(&T, m, n, rowptr, col)) return -2;
  int32_t *rp, *cl;
  int32_t nv = window_csr(&T, w, w_eps, &rp, &cl);
  if (nv >= 0) {
    memcpy(rowptr_out, rp, sizeof(int32_t) * ((size_t)w * m + 1));
    memcpy(col_out, cl, sizeof(int32_t) * (size_t)rp[w * m]);
    free(rp);
    free(cl);
  }
  tanner_free(&T);
  return nv;
}

/* ------------------------------------------------------------------------
 * Pins only: the discrete bit-centric machine (SM "Setup and algorithm"),
 * in double precision with libm tanh/atanh.
 *
 * Iteration i (from the state of iteration i-1; all updates use old values):
 *   check-to-bit   m^_{c->v} = 2 (-1)^{s_c + d_c} atanh(prod tanh(m_{w->c}/2))
 *                  (for d_c = 2 this is (-1)^{s_c} m_{w->c});
 *   bit-to-check   m^_{v->c} = pi_v + sum_{c' != c} m_{c'->v};
 *   beliefs        L^_v = pi_v + sum_c m_{c->v};
 *   feedback       f_v = 1[L^_v > 0]; s_c ^= XOR_{v in N(c)} f_v;
 *   LLR switch     pi_v, m^_{v->c}, m^_{c->v} multiplied by (-1)^{f_v}.
 * Messages and pi start at 0 and log(q/(1-q)). Records e^{(i)} = e0 ^ z^{(i)}
 * for i = 1..iters into e_trace [iters][n] and the beliefs L^ into L_trace.
 * ---------------------------------------------------------------------- */
int32_t orc_bitcentric_machine(int32_t m, int32_t n, const int32_t* rowptr, const int32_t* col,
                               double q, const uint8_t* e0, int32_t iters, uint8_t* e_trace,
                               double* L_trace, int32_t* iclr_out) {
  tanner T;
  if (tanner_init(&T, m, n, rowptr, col)) return -2;
  const int32_t E = T.E;
  double* mvc = (double*)calloc((size_t)E + 1, sizeof(double));
  double* mcv = (double*)calloc((size_t)E + 1, sizeof(double));
  double* nvc = (double*)calloc((size_t)E + 1, sizeof(double));
  double* ncv = (double*)calloc((size_t)E + 1, sizeof(double));
  double* piv = (double*)malloc(sizeof(double) * ((size_t)n + 1));
  uint8_t* s = (uint8_t*)malloc((size_t)m + 1);
  uint8_t* z = (uint8_t*)calloc((size_t)n + 1, 1);
  uint8_t* f = (uint8_t*)calloc((size_t)n + 1, 1);
  double pi0 = log(q / (1.0 - q));
  for (int32_t v = 0; v < n; ++v) piv[v] = pi0;
  orc_syndrome(m, n, rowptr, col, e0, 1, s);
  int any = 0;
  for (int32_t c = 0; c < m; ++c) any |= s[c];
  *iclr_out = any ? -1 : 0;
  for (int32_t it = 1; it <= iters; ++it) {
    for (int32_t c = 0; c < m; ++c) {
      int32_t b = rowptr[c], dc = rowptr[c + 1] - b;
      double sg = ((s[c] + dc) & 1) ? -1.0 : 1.0;
      for (int32_t j = 0; j < dc; ++j) {
        double prod = 1.0;
        for (int32_t i = 0; i < dc; ++i)
          if (i != j) prod *= tanh(mvc[b + i] / 2.0);
        ncv[b + j] = (dc == 2) ? sg * mvc[b + (1 - j)] : sg * 2.0 * atanh(prod);
      }
    }
    for (int32_t v = 0; v < n; ++v) {
      int32_t b = T.vptr[v], dv = T.vptr[v + 1] - b;
      double Lh = piv[v];
      for (int32_t i = 0; i < dv; ++i) Lh += mcv[T.vedge[b + i]];
      for (int32_t j = 0; j < dv; ++j) {
        double acc = piv[v];
        for (int32_t i = 0; i < dv; ++i)
          if (i != j) acc += mcv[T.vedge[b + i]];
        nvc[T.vedge[b + j]] = acc;
      }
      f[v] = Lh > 0.0;
      if (L_trace) L_trace[(size_t)(it - 1) * n + v] = Lh;
    }
    for (int32_t c = 0; c < m; ++c)
      for (int32_t k = rowptr[c]; k < rowptr[c + 1]; ++k) s[c] ^= f[col[k]];
    for (int32_t v = 0; v < n; ++v) {
      z[v] ^= f[v];
      double g = f[v] ? -1.0 : 1.0;
      piv[v] *= g;
      for (int32_t i = T.vptr[v]; i < T.vptr[v + 1]; ++i) {
        int32_t e = T.vedge[i];
        nvc[e] *= g;
        ncv[e] *= g;
      }
      if (e_trace) e_trace[(size_t)(it - 1) * n + v] = (uint8_t)(e0[v] ^ z[v]);
    }
    memcpy(mvc, nvc, sizeof(double) * (size_t)E);
    memcpy(mcv, ncv, sizeof(double) * (size_t)E);
    any = 0;
    for (int32_t c = 0; c < m; ++c) any |= s[c];
    if (!any && *iclr_out < 0) *iclr_out = it;
  }
  free(mvc); free(mcv); free(nvc); free(ncv); free(piv); free(s); free(z); free(f);
  tanner_free(&T);
  return 0;
}

/* Elementwise helpers so the tests can pin the FP32 functions on many points. */
void orc_vec_exp_neg(const float* x, int32_t k, float* y) { for (int32_t i = 0; i < k; ++i) y[i] = orc_exp_neg(x[i]); }
void orc_vec_log1p_unit(const float* x, int32_t k, float* y) { for (int32_t i = 0; i < k; ++i) y[i] = orc_log1p_unit(x[i]); }
void orc_vec_boxplus(const float* a, const float* b, int32_t k, float* y) { for (int32_t i = 0; i < k; ++i) y[i] = orc_boxplus(a[i], b[i]); }
void orc_vec_philox(const uint32_t* ctr, const uint32_t* key, int32_t k, uint32_t* out) {
  for (int32_t i = 0; i < k; ++i) orc_philox4x32_10(ctr + 4 * (size_t)i, key + 2 * (size_t)i, out + 4 * (size_t)i);
}
