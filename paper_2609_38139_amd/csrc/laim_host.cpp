// laim_host.cpp -- host side of the C ABI: code layout, logical basis,
// parameter checks and dispatch of the kernels.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "laim_internal.h"

namespace laim {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

laim_status hip_fail(hipError_t e, const char* what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return LAIM_EHIP;
}

uint64_t bernoulli_bound(double p) {
  if (!(p > 0.0)) return 0;
  if (p >= 1.0) return (uint64_t)1 << 32;
  return (uint64_t)floor(p * 4294967296.0);
}

laim_status resolve_params(const laim_decode_params* p, KParams* kp) {
  if (!p) {
    set_error("params is NULL");
    return LAIM_EINVAL;
  }
  if (p->bp != 0 && p->bp != 1) {
    set_error("bp must be 0 (min-sum) or 1 (sum-product)");
    return LAIM_EINVAL;
  }
  if (!(p->q > 0.0 && p->q < 1.0)) {
    set_error("decoder prior q must lie in (0, 1)");
    return LAIM_EINVAL;
  }
  if (!(p->clamp > 0.0f) || !(p->alpha > 0.0f)) {
    set_error("clamp and alpha must be positive");
    return LAIM_EINVAL;
  }
  if (p->iters < 0 || p->rounds < 0 || p->rounds > (1 << 27)) {
    set_error("iters must be >= 0 and rounds in [0, 2^27]");
    return LAIM_EINVAL;
  }
  if (p->gauge != 0) {
    set_error("gauge = 1 (the bit-centric LLR switch) is not part of the check-centric machine");
    return LAIM_EUNSUP;
  }
  if (p->conflict < LAIM_CONFLICT_OR || p->conflict > LAIM_CONFLICT_SEQUENTIAL) {
    set_error("conflict must be LAIM_CONFLICT_OR, _XOR or _SEQUENTIAL");
    return LAIM_EINVAL;
  }
  if (p->move != LAIM_MOVE_SINGLE && p->move != LAIM_MOVE_MULTI) {
    set_error("move must be LAIM_MOVE_SINGLE or LAIM_MOVE_MULTI");
    return LAIM_EINVAL;
  }
  if (p->move == LAIM_MOVE_MULTI && p->conflict == LAIM_CONFLICT_SEQUENTIAL) {
    set_error("multi-qubit moves combine by OR or XOR only");
    return LAIM_EUNSUP;
  }
  kp->bp = p->bp;
  kp->alpha = p->alpha;
  kp->pi = (float)log(p->q / (1.0 - p->q));
  kp->clamp = p->clamp;
  kp->iters = p->iters;
  kp->rounds = p->rounds;
  kp->mask_bound = bernoulli_bound(p->mask_density);
  kp->evidence = p->evidence ? 1 : 0;
  kp->retire = p->retire ? 1 : 0;
  kp->seed = p->seed;
  kp->conflict = p->conflict;
  kp->skip = p->skip_fixed ? 1 : 0;
  kp->move = p->move;
  return LAIM_OK;
}

// ------------------------------------------------------------------ GF(2)
// Dense bit-packed rows; elimination by row operations.
struct Bits {
  int32_t n = 0, words = 0;
  std::vector<uint64_t> a;  // rows x words
  int32_t rows() const { return words ? (int32_t)(a.size() / words) : 0; }
  uint64_t* row(int32_t r) { return a.data() + (size_t)r * words; }
  const uint64_t* row(int32_t r) const { return a.data() + (size_t)r * words; }
};

static Bits pack_csr(int32_t rows, int32_t n, const int32_t* rp, const int32_t* col) {
  Bits b;
  b.n = n;
  b.words = (n + 63) / 64;
  b.a.assign((size_t)rows * b.words, 0);
  for (int32_t r = 0; r < rows; ++r)
    for (int32_t k = rp[r]; k < rp[r + 1]; ++k)
      b.row(r)[col[k] >> 6] ^= (uint64_t)1 << (col[k] & 63);
  return b;
}

static inline bool bit(const uint64_t* r, int32_t c) { return (r[c >> 6] >> (c & 63)) & 1u; }
static inline void xor_row(uint64_t* d, const uint64_t* s, int32_t from_word, int32_t words) {
  for (int32_t k = from_word; k < words; ++k) d[k] ^= s[k];
}

// Reduced row echelon form in place; returns the pivot columns.
static std::vector<int32_t> rref(Bits& b) {
  std::vector<int32_t> piv;
  const int32_t R = b.rows();
  int32_t r = 0;
  for (int32_t c = 0; c < b.n && r < R; ++c) {
    int32_t p = -1;
    for (int32_t i = r; i < R; ++i)
      if (bit(b.row(i), c)) {
        p = i;
        break;
      }
    if (p < 0) continue;
    if (p != r) std::swap_ranges(b.row(p), b.row(p) + b.words, b.row(r));
    for (int32_t i = 0; i < R; ++i)
      if (i != r && bit(b.row(i), c)) xor_row(b.row(i), b.row(r), c >> 6, b.words);
    piv.push_back(c);
    ++r;
  }
  b.a.resize((size_t)r * b.words);
  return piv;
}

// Echelon basis with insertion (for independence tests modulo a span).
struct Echelon {
  int32_t words;
  std::vector<std::vector<uint64_t>> rows;
  std::vector<int32_t> piv;  // leading column of each row, ascending
  explicit Echelon(int32_t w) : words(w) {}
  // Reduces x; returns true and inserts it if it is independent.
  bool insert(std::vector<uint64_t> x) {
    for (size_t i = 0; i < rows.size(); ++i)
      if (bit(x.data(), piv[i])) xor_row(x.data(), rows[i].data(), piv[i] >> 6, words);
    int32_t lead = -1;
    for (int32_t k = 0; k < words && lead < 0; ++k)
      if (x[k]) lead = k * 64 + __builtin_ctzll(x[k]);
    if (lead < 0) return false;
    // keep rows sorted by pivot so that reduction in order stays valid
    size_t pos = std::lower_bound(piv.begin(), piv.end(), lead) - piv.begin();
    // eliminate the new pivot from later rows is not needed: reduction goes
    // in ascending pivot order and rows have zeros before their pivot
    rows.insert(rows.begin() + pos, std::move(x));
    piv.insert(piv.begin() + pos, lead);
    return true;
  }
};

// Basis of ker(G) modulo row(H): k vectors (dense 0/1 rows).
static laim_status logical_basis(int32_t m, int32_t n, const int32_t* hrp, const int32_t* hc,
                                 int32_t mg, const int32_t* grp, const int32_t* gc,
                                 std::vector<std::vector<uint8_t>>* out) {
  if (n > 20480) {
    set_error("logical basis by elimination is limited to n <= 20480 (n = %d); pass logicals", n);
    return LAIM_EUNSUP;
  }
  Bits G = pack_csr(mg, n, grp, gc);
  std::vector<int32_t> gp = rref(G);
  Bits H = pack_csr(m, n, hrp, hc);
  Bits Hr = H;
  std::vector<int32_t> hp = rref(Hr);
  const int32_t k = n - (int32_t)hp.size() - (int32_t)gp.size();
  out->clear();
  if (k <= 0) return LAIM_OK;
  Echelon E(H.words);
  for (int32_t i = 0; i < Hr.rows(); ++i) {
    std::vector<uint64_t> r(Hr.row(i), Hr.row(i) + Hr.words);
    E.insert(std::move(r));
  }
  std::vector<char> is_piv(n, 0);
  for (int32_t c : gp) is_piv[c] = 1;
  for (int32_t f = 0; f < n && (int32_t)out->size() < k; ++f) {
    if (is_piv[f]) continue;
    // kernel vector of the RREF of G with free column f set
    std::vector<uint64_t> x(H.words, 0);
    x[f >> 6] |= (uint64_t)1 << (f & 63);
    for (size_t i = 0; i < gp.size(); ++i)
      if (bit(G.row((int32_t)i), f)) x[gp[i] >> 6] ^= (uint64_t)1 << (gp[i] & 63);
    std::vector<uint64_t> keep = x;
    if (E.insert(std::move(x))) {
      std::vector<uint8_t> v(n, 0);
      for (int32_t c = 0; c < n; ++c) v[c] = bit(keep.data(), c) ? 1 : 0;
      out->push_back(std::move(v));
    }
  }
  if ((int32_t)out->size() != k) {
    set_error("internal: found %zu logicals, expected %d", out->size(), k);
    return LAIM_EINVAL;
  }
  return LAIM_OK;
}

static laim_status check_csr(const char* what, int32_t rows, int32_t n, const int32_t* rp,
                             const int32_t* col) {
  if (rows < 0 || (rows > 0 && !rp)) {
    set_error("%s: bad row count or NULL row pointers", what);
    return LAIM_EINVAL;
  }
  if (rows == 0) return LAIM_OK;
  if (rp[0] != 0) {
    set_error("%s: rowptr[0] must be 0", what);
    return LAIM_EINVAL;
  }
  for (int32_t r = 0; r < rows; ++r) {
    if (rp[r + 1] < rp[r]) {
      set_error("%s: row pointers must not decrease", what);
      return LAIM_EINVAL;
    }
    for (int32_t k = rp[r]; k < rp[r + 1]; ++k) {
      if (!col || col[k] < 0 || col[k] >= n) {
        set_error("%s: column index out of range in row %d", what, r);
        return LAIM_EINVAL;
      }
      if (k > rp[r] && col[k] <= col[k - 1]) {
        set_error("%s: columns must be strictly ascending in row %d", what, r);
        return LAIM_EINVAL;
      }
    }
  }
  return LAIM_OK;
}

// even overlap of every row of A with every row of B (sparse)
static bool rows_commute(int32_t ma, int32_t n, const int32_t* arp, const int32_t* ac, int32_t mb,
                         const int32_t* brp, const int32_t* bc) {
  if (ma == 0 || mb == 0) return true;
  std::vector<std::vector<int32_t>> bcol(n);
  for (int32_t r = 0; r < mb; ++r)
    for (int32_t k = brp[r]; k < brp[r + 1]; ++k) bcol[bc[k]].push_back(r);
  std::vector<uint8_t> par(mb, 0);
  std::vector<int32_t> touched;
  for (int32_t r = 0; r < ma; ++r) {
    touched.clear();
    for (int32_t k = arp[r]; k < arp[r + 1]; ++k)
      for (int32_t b : bcol[ac[k]]) {
        if (!par[b]) touched.push_back(b);
        par[b] ^= 1;
        if (!par[b]) touched.push_back(b);
      }
    bool bad = false;
    for (int32_t b : touched) {
      if (par[b]) bad = true;
      par[b] = 0;
    }
    if (bad) return false;
  }
  return true;
}

}  // namespace laim

using namespace laim;

// ===================================================================== ABI
extern "C" {

const char* laim_last_error(void) { return g_last_error.c_str(); }
int32_t laim_version(void) { return 2; }

laim_status laim_host_logicals(int32_t m, int32_t n, const int32_t* h_rowptr, const int32_t* h_col,
                               int32_t mg, const int32_t* g_rowptr, const int32_t* g_col,
                               int32_t kmax, uint8_t* out, int32_t* k_out) {
  laim_status st;
  if (m < 1 || n < 1) {
    set_error("m and n must be >= 1");
    return LAIM_EINVAL;
  }
  if ((st = check_csr("H", m, n, h_rowptr, h_col)) != LAIM_OK) return st;
  if ((st = check_csr("G", mg, n, g_rowptr, g_col)) != LAIM_OK) return st;
  std::vector<std::vector<uint8_t>> L;
  if ((st = logical_basis(m, n, h_rowptr, h_col, mg, g_rowptr, g_col, &L)) != LAIM_OK) return st;
  if (k_out) *k_out = (int32_t)L.size();
  if (out)
    for (int32_t i = 0; i < (int32_t)L.size() && i < kmax; ++i)
      memcpy(out + (size_t)i * n, L[i].data(), (size_t)n);
  return LAIM_OK;
}

// The 2D toric layout (DevCode::tile_*): m = L^2 checks of degree 4 on
// n = 2 m qubits of degree 2, L a multiple of 4, where check i L + j shares
// exactly one qubit with each of (i, j -/+ 1) and (i -/+ 1, j) (indices mod L)
// and those four qubits are its row. Fills the tiled variant's tables.
static bool toric_tiles(int32_t m, int32_t n, int32_t dcmax, const std::vector<int32_t>& chk_deg,
                        const std::vector<int32_t>& chk_var, const std::vector<int32_t>& vdeg,
                        std::vector<int32_t>* tchk, std::vector<int32_t>* tjo,
                        std::vector<int32_t>* tword, int32_t* Lout) {
  const int32_t L = (int32_t)lround(sqrt((double)m));
  *Lout = L;
  if (dcmax != 4 || L < 4 || L % 4 != 0 || L * L != m || n != 2 * m) return false;
  for (int32_t c = 0; c < m; ++c)
    if (chk_deg[c] != 4) return false;
  for (int32_t v = 0; v < n; ++v)
    if (vdeg[v] != 2) return false;
  // jo[4 c + g]: the row slot of the qubit check c shares with its neighbour
  // in direction g (0 left, 1 right, 2 up, 3 down)
  std::vector<int32_t> jo((size_t)m * 4);
  for (int32_t i = 0; i < L; ++i)
    for (int32_t j = 0; j < L; ++j) {
      const int32_t c = i * L + j;
      const int32_t nb[4] = {i * L + (j + L - 1) % L, i * L + (j + 1) % L, ((i + L - 1) % L) * L + j,
                             ((i + 1) % L) * L + j};
      uint32_t used = 0u;
      for (int g = 0; g < 4; ++g) {
        int32_t slot = -1, count = 0;
        for (int s = 0; s < 4; ++s)
          for (int s2 = 0; s2 < 4; ++s2)
            if (chk_var[(size_t)c * 4 + s] == chk_var[(size_t)nb[g] * 4 + s2]) {
              ++count;
              slot = s;
            }
        if (count != 1 || (used >> slot) & 1u) return false;
        used |= 1u << slot;
        jo[(size_t)c * 4 + g] = slot;
      }
    }
  const int32_t nt = m / 8, tw = L / 4;
  tchk->assign((size_t)m, 0);
  tjo->assign((size_t)m * 4, 0);
  tword->assign((size_t)m * 4, 0);
  for (int32_t t = 0; t < nt; ++t)
    for (int32_t k = 0; k < 8; ++k) {
      const int32_t c = (2 * (t / tw) + (k >> 2)) * L + 4 * (t % tw) + (k & 3);
      const int32_t vc = t + k * nt;
      (*tchk)[vc] = c;
      for (int g = 0; g < 4; ++g) {
        const int32_t s = jo[(size_t)c * 4 + g];
        (*tjo)[(size_t)vc * 4 + g] = s;
        (*tword)[(size_t)c * 4 + s] = resident_msg_word(4, vc, g);
      }
    }
  return true;
}

laim_status laim_build_tanner_ex(int32_t m, int32_t n, const int32_t* h_rowptr,
                                 const int32_t* h_col, int32_t mg, const int32_t* g_rowptr,
                                 const int32_t* g_col, int32_t kl, const int32_t* l_rowptr,
                                 const int32_t* l_col, int32_t device, laim_code** out) {
  if (!out) {
    set_error("out is NULL");
    return LAIM_EINVAL;
  }
  *out = nullptr;
  if (m < 1 || n < 1) {
    set_error("m and n must be >= 1");
    return LAIM_EINVAL;
  }
  laim_status st;
  if ((st = check_csr("H", m, n, h_rowptr, h_col)) != LAIM_OK) return st;
  if ((st = check_csr("G", mg, n, g_rowptr, g_col)) != LAIM_OK) return st;
  if (kl >= 0 && (st = check_csr("logicals", kl, n, l_rowptr, l_col)) != LAIM_OK) return st;
  const int32_t E = h_rowptr[m];
  int32_t dcmax = 0;
  for (int32_t c = 0; c < m; ++c) dcmax = std::max(dcmax, h_rowptr[c + 1] - h_rowptr[c]);
  std::vector<int32_t> vdeg(n, 0);
  for (int32_t e = 0; e < E; ++e) vdeg[h_col[e]]++;
  int32_t dvmax = 0, dvmin = 1 << 30, dcmin = 1 << 30;
  for (int32_t v = 0; v < n; ++v) {
    dvmax = std::max(dvmax, vdeg[v]);
    dvmin = std::min(dvmin, vdeg[v]);
  }
  for (int32_t c = 0; c < m; ++c) dcmin = std::min(dcmin, h_rowptr[c + 1] - h_rowptr[c]);
  if (dvmin < 1) {
    set_error("every qubit must lie in at least one check");
    return LAIM_EINVAL;
  }
  if (dcmax > kMaxCheckDegree || dvmax > kMaxQubitDegree) {
    set_error("check degree %d / qubit degree %d above the supported %d / %d", dcmax, dvmax,
              kMaxCheckDegree, kMaxQubitDegree);
    return LAIM_EUNSUP;
  }
  if (!rows_commute(m, n, h_rowptr, h_col, mg, g_rowptr, g_col)) {
    set_error("H G^T != 0: G must commute with H");
    return LAIM_EINVAL;
  }
  std::vector<std::vector<uint8_t>> logi;
  if (kl < 0) {
    if ((st = logical_basis(m, n, h_rowptr, h_col, mg, g_rowptr, g_col, &logi)) != LAIM_OK)
      return st;
  } else {
    if (!rows_commute(kl, n, l_rowptr, l_col, mg, g_rowptr, g_col)) {
      set_error("a given logical has odd overlap with a row of G");
      return LAIM_EINVAL;
    }
    for (int32_t i = 0; i < kl; ++i) {
      std::vector<uint8_t> v(n, 0);
      for (int32_t k = l_rowptr[i]; k < l_rowptr[i + 1]; ++k) v[l_col[k]] = 1;
      logi.push_back(std::move(v));
    }
  }
  const int32_t k = (int32_t)logi.size();
  const int32_t kw = (k + 31) / 32;

  // ---- host tables
  std::vector<int32_t> chk_var((size_t)m * dcmax, -1), chk_deg(m);
  for (int32_t c = 0; c < m; ++c) {
    chk_deg[c] = h_rowptr[c + 1] - h_rowptr[c];
    for (int32_t j = 0; j < chk_deg[c]; ++j) chk_var[(size_t)c * dcmax + j] = h_col[h_rowptr[c] + j];
  }
  std::vector<int32_t> var_edge((size_t)n * dvmax, -1), fill(n, 0);
  for (int32_t c = 0; c < m; ++c)  // ascending c: each qubit's list ascends
    for (int32_t j = 0; j < chk_deg[c]; ++j) {
      const int32_t v = chk_var[(size_t)c * dcmax + j];
      var_edge[(size_t)v * dvmax + fill[v]++] = pack_edge(c, j);
    }
  const int32_t pw = std::max(dvmax - 1, 1);
  std::vector<int32_t> partner((size_t)m * dcmax * pw, -1);
  for (int32_t c = 0; c < m; ++c)
    for (int32_t j = 0; j < chk_deg[c]; ++j) {
      const int32_t v = chk_var[(size_t)c * dcmax + j];
      int32_t p = 0;
      for (int32_t q = 0; q < vdeg[v]; ++q) {
        const int32_t e = var_edge[(size_t)v * dvmax + q];
        if (edge_check(e) == c) continue;
        partner[((size_t)c * dcmax + j) * pw + p++] = e;
      }
    }
  std::vector<uint32_t> lcol((size_t)n * std::max(kw, 1), 0u);
  for (int32_t i = 0; i < k; ++i)
    for (int32_t v = 0; v < n; ++v)
      if (logi[i][v]) lcol[(size_t)v * kw + (i >> 5)] |= 1u << (i & 31);
  std::vector<float> thr(dcmax + 1);
  for (int32_t d = 0; d <= dcmax; ++d) thr[d] = (d <= 1) ? INFINITY : (float)(-log((double)(d - 1)));

  std::vector<int32_t> tile_chk, tile_jo, tile_word;
  int32_t tile_L = 0;
  const bool tiled =
      toric_tiles(m, n, dcmax, chk_deg, chk_var, vdeg, &tile_chk, &tile_jo, &tile_word, &tile_L);

  // ---- one device allocation
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t b_cv = al(chk_var.size() * 4), b_cd = al((size_t)m * 4), b_vd = al((size_t)n * 4),
               b_ve = al(var_edge.size() * 4), b_pa = al(partner.size() * 4),
               b_lc = al(lcol.size() * 4), b_th = al(thr.size() * 4),
               b_tc = al(tile_chk.size() * 4), b_tj = al(tile_jo.size() * 4),
               b_tw = al(tile_word.size() * 4);
  const size_t total = b_cv + b_cd + b_vd + b_ve + b_pa + b_lc + b_th + b_tc + b_tj + b_tw;
  int prev = 0;
  (void)hipGetDevice(&prev);
  hipError_t he = hipSetDevice(device);
  if (he != hipSuccess) return hip_fail(he, "hipSetDevice");
  void* dmem = nullptr;
  he = hipMalloc(&dmem, total);
  if (he != hipSuccess) {
    (void)hipSetDevice(prev);
    set_error("hipMalloc of %zu bytes for the code tables failed", total);
    return LAIM_ENOMEM;
  }
  char* p = (char*)dmem;
  size_t off = 0;
  auto up = [&](const void* src, size_t bytes, size_t span) -> void* {
    void* d = p + off;
    if (bytes) he = (he == hipSuccess) ? hipMemcpy(d, src, bytes, hipMemcpyHostToDevice) : he;
    off += span;
    return d;
  };
  he = hipSuccess;
  laim_code* code = new (std::nothrow) laim_code();
  if (!code) {
    (void)hipFree(dmem);
    (void)hipSetDevice(prev);
    set_error("out of host memory");
    return LAIM_ENOMEM;
  }
  DevCode& d = code->dev;
  d.m = m;
  d.n = n;
  d.E = E;
  d.dcmax = dcmax;
  d.dvmax = dvmax;
  d.k = k;
  d.kw = kw;
  d.regular = (dcmin == dcmax && dvmin == dvmax) ? 1 : 0;
  d.chk_var = (const int32_t*)up(chk_var.data(), chk_var.size() * 4, b_cv);
  d.chk_deg = (const int32_t*)up(chk_deg.data(), (size_t)m * 4, b_cd);
  d.var_deg = (const int32_t*)up(vdeg.data(), (size_t)n * 4, b_vd);
  d.var_edge = (const int32_t*)up(var_edge.data(), var_edge.size() * 4, b_ve);
  d.partner = (const int32_t*)up(partner.data(), partner.size() * 4, b_pa);
  d.lcol = (const uint32_t*)up(lcol.data(), lcol.size() * 4, b_lc);
  d.thr = (const float*)up(thr.data(), thr.size() * 4, b_th);
  d.tile_chk = tiled ? (const int32_t*)up(tile_chk.data(), tile_chk.size() * 4, b_tc) : nullptr;
  d.tile_jo = tiled ? (const int32_t*)up(tile_jo.data(), tile_jo.size() * 4, b_tj) : nullptr;
  d.tile_word = tiled ? (const int32_t*)up(tile_word.data(), tile_word.size() * 4, b_tw) : nullptr;
  d.tile_L = tiled ? tile_L : 0;
  (void)hipSetDevice(prev);
  if (he != hipSuccess) {
    (void)hipFree(dmem);
    delete code;
    return hip_fail(he, "uploading code tables");
  }
  code->device = device;
  code->m = m;
  code->n = n;
  code->E = E;
  code->dcmax = dcmax;
  code->dvmax = dvmax;
  code->k = k;
  code->h_rowptr.assign(h_rowptr, h_rowptr + m + 1);
  code->h_col.assign(h_col, h_col + E);
  code->logicals.assign((size_t)k * n, 0);
  for (int32_t i = 0; i < k; ++i) memcpy(code->logicals.data() + (size_t)i * n, logi[i].data(), n);
  code->dev_mem = dmem;
  code->has_cfg[0] = code->has_cfg[1] = false;
  *out = code;
  return LAIM_OK;
}

laim_status laim_build_tanner(int32_t m, int32_t n, const int32_t* h_rowptr, const int32_t* h_col,
                              int32_t mg, const int32_t* g_rowptr, const int32_t* g_col,
                              int32_t device, laim_code** out) {
  return laim_build_tanner_ex(m, n, h_rowptr, h_col, mg, g_rowptr, g_col, -1, nullptr, nullptr,
                              device, out);
}

void laim_free_code(laim_code* code) {
  if (!code) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(code->device);
  (void)hipFree(code->dev_mem);
  (void)hipSetDevice(prev);
  delete code;
}

laim_status laim_code_info(const laim_code* code, int32_t* m, int32_t* n, int32_t* E, int32_t* k,
                           int32_t* dc_max, int32_t* dv_max) {
  if (!code) {
    set_error("code is NULL");
    return LAIM_EINVAL;
  }
  if (m) *m = code->m;
  if (n) *n = code->n;
  if (E) *E = code->E;
  if (k) *k = code->k;
  if (dc_max) *dc_max = code->dcmax;
  if (dv_max) *dv_max = code->dvmax;
  return LAIM_OK;
}

laim_status laim_code_logicals(const laim_code* code, uint8_t* out) {
  if (!code || (!out && code->k > 0)) {
    set_error("code or out is NULL");
    return LAIM_EINVAL;
  }
  if (code->k) memcpy(out, code->logicals.data(), code->logicals.size());
  return LAIM_OK;
}

// RAII device switch for calls on a code's device.
struct DeviceGuard {
  int prev = 0;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    (void)hipGetDevice(&prev);
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() { (void)hipSetDevice(prev); }
};

laim_status laim_sample_noise(const laim_code* code, double p, uint64_t seed, uint64_t shot0,
                              int32_t nshots, uint8_t* e_out, laim_stream stream) {
  if (!code || nshots < 0 || (nshots > 0 && !e_out)) {
    set_error("laim_sample_noise: bad arguments");
    return LAIM_EINVAL;
  }
  if (p != p) {
    set_error("p is NaN");
    return LAIM_EINVAL;
  }
  DeviceGuard g(code->device);
  hipError_t e = launch_noise(code->dev, bernoulli_bound(p), seed, shot0, nshots, e_out,
                              (hipStream_t)stream);
  return e == hipSuccess ? LAIM_OK : hip_fail(e, "noise kernel");
}

laim_status laim_syndrome(const laim_code* code, const uint8_t* e, int32_t nshots, uint8_t* s_out,
                          laim_stream stream) {
  if (!code || nshots < 0 || (nshots > 0 && (!e || !s_out))) {
    set_error("laim_syndrome: bad arguments");
    return LAIM_EINVAL;
  }
  DeviceGuard g(code->device);
  hipError_t er = launch_syndrome(code->dev, e, nshots, s_out, (hipStream_t)stream);
  return er == hipSuccess ? LAIM_OK : hip_fail(er, "syndrome kernel");
}

laim_status laim_logical_failure(const laim_code* code, const uint8_t* e0, const uint8_t* z,
                                 int32_t nshots, uint8_t* fail_out, laim_stream stream) {
  if (!code || nshots < 0 || (nshots > 0 && (!e0 || !z || !fail_out))) {
    set_error("laim_logical_failure: bad arguments");
    return LAIM_EINVAL;
  }
  if (code->dev.kw > 64) {
    set_error("more than 2048 logicals are not supported");
    return LAIM_EUNSUP;
  }
  DeviceGuard g(code->device);
  hipError_t er = launch_failure(code->dev, e0, z, nshots, fail_out, (hipStream_t)stream);
  return er == hipSuccess ? LAIM_OK : hip_fail(er, "failure kernel");
}

static int resolve_form(const laim_code* code, int bp, bool seq, bool reg2, int form, ResidentShape* sh) {
  const laim_resident_cfg* want = code->has_cfg[bp] ? &code->cfg[bp] : nullptr;
  if (form == LAIM_FORM_STREAM) return LAIM_FORM_STREAM;
  const bool ok = resident_shape(code->dev, bp, want, sh, code->device, seq, reg2);
  if (form == LAIM_FORM_RESIDENT) return ok ? LAIM_FORM_RESIDENT : -1;
  return ok ? LAIM_FORM_RESIDENT : LAIM_FORM_STREAM;
}

laim_status laim_resident_variant(const laim_code* code, const laim_decode_params* params,
                                  const laim_resident_cfg* cfg, int32_t* dc, int32_t* dv,
                                  int32_t* checks_per_thread, int32_t* tiled) {
  if (!code || !params) {
    set_error("laim_resident_variant: bad arguments");
    return LAIM_EINVAL;
  }
  KParams kp;
  laim_status st = resolve_params(params, &kp);
  if (st != LAIM_OK) return st;
  if (kp.bp == 0 && kp.alpha > 1.0f) {
    set_error("the resident min-sum form needs alpha <= 1");
    return LAIM_EUNSUP;
  }
  const bool seq = kp.conflict == kConflictSequential;
  const laim_resident_cfg* want = cfg ? cfg : (code->has_cfg[kp.bp] ? &code->cfg[kp.bp] : nullptr);
  ResidentShape sh;
  if (!resident_shape(code->dev, kp.bp, want, &sh, code->device, seq, reg_dv2_ok(kp))) return LAIM_EUNSUP;
  if (dc) *dc = sh.dc;
  if (dv) *dv = sh.dv;
  if (checks_per_thread) *checks_per_thread = sh.cpt;
  if (tiled) *tiled = sh.tile;
  return LAIM_OK;
}

size_t laim_workspace_bytes(const laim_code* code, const laim_decode_params* params,
                            int32_t nshots, int32_t form) {
  if (!code || !params || nshots < 0) return 0;
  ResidentShape sh;
  const bool seq = params->conflict == LAIM_CONFLICT_SEQUENTIAL;
  KParams kp;
  if (resolve_params(params, &kp) != LAIM_OK) return 0;
  int f = resolve_form(code, kp.bp, seq, reg_dv2_ok(kp), form, &sh);
  if (params->bp == 0 && params->alpha > 1.0f) f = (form == LAIM_FORM_RESIDENT) ? -1 : LAIM_FORM_STREAM;
  if (f == LAIM_FORM_RESIDENT) return resident_workspace_bytes();
  if (f == LAIM_FORM_STREAM) return stream_workspace_bytes(code->dev, nshots, seq);
  return 0;
}

}  // extern "C"

namespace laim {

laim_status decode_common(const laim_code* code, const laim_decode_params* params,
                                 const uint8_t* e0, uint64_t shot0, int32_t nshots, void* ws,
                                 size_t ws_bytes, uint8_t* z_out, uint8_t* s_out, int32_t* tclr_out,
                                 float* L_out, int32_t* sweeps_out, uint8_t* fail_out, int32_t form,
                                 const laim_resident_cfg* cfg, laim_stream stream) {
  if (!code || nshots < 0 || (nshots > 0 && (!e0 || !z_out || !s_out || !tclr_out))) {
    set_error("laim_decode_rounds: bad arguments");
    return LAIM_EINVAL;
  }
  KParams kp;
  laim_status st = resolve_params(params, &kp);
  if (st != LAIM_OK) return st;
  if (form < LAIM_FORM_AUTO || form > LAIM_FORM_STREAM) {
    set_error("unknown form %d", form);
    return LAIM_EINVAL;
  }
  if (fail_out && code->dev.kw > 64) {
    set_error("more than 2048 logicals are not supported");
    return LAIM_EUNSUP;
  }
  if (nshots == 0) return LAIM_OK;
  const bool seq = kp.conflict == kConflictSequential;
  ResidentShape sh;
  int f;
  // The resident min-sum kernel relies on alpha <= 1 (its outputs cannot
  // reach the clamp); other scales run in the stream form.
  const bool resident_ok = !(kp.bp == 0 && kp.alpha > 1.0f);
  if (cfg) {
    if (!resident_ok) {
      set_error("the resident min-sum form needs alpha <= 1");
      return LAIM_EUNSUP;
    }
    if (!resident_shape(code->dev, kp.bp, cfg, &sh, code->device, seq, reg_dv2_ok(kp))) return LAIM_EINVAL;
    f = LAIM_FORM_RESIDENT;
  } else if (!resident_ok) {
    if (form == LAIM_FORM_RESIDENT) {
      set_error("the resident min-sum form needs alpha <= 1");
      return LAIM_EUNSUP;
    }
    f = LAIM_FORM_STREAM;
  } else {
    f = resolve_form(code, kp.bp, seq, reg_dv2_ok(kp), form, &sh);
    if (f < 0) {
      set_error("the code cannot run in the resident form (a shot's state exceeds the LDS or its "
                "degrees have no compiled variant)");
      return LAIM_EUNSUP;
    }
  }
  const size_t need = (f == LAIM_FORM_RESIDENT) ? resident_workspace_bytes()
                                                : stream_workspace_bytes(code->dev, nshots, seq);
  if (!ws || ws_bytes < need) {
    set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
    return LAIM_ENOMEM;
  }
  if (((uintptr_t)ws) % 256) {
    set_error("workspace must be 256-byte aligned");
    return LAIM_EINVAL;
  }
  DeviceGuard g(code->device);
  hipError_t er;
  // the resident kernel folds the failure test into the launch for codes
  // with at most 128 logicals; otherwise it runs as its own kernel after
  const bool fused_fail = f == LAIM_FORM_RESIDENT && code->dev.kw <= 4;
  if (f == LAIM_FORM_RESIDENT) {
    er = launch_resident(code->dev, kp, sh, e0, shot0, nshots, ws, z_out, s_out, tclr_out, L_out,
                         fused_fail ? fail_out : nullptr, sweeps_out, (hipStream_t)stream);
  } else {
    er = launch_stream(code->dev, kp, e0, shot0, nshots, ws, z_out, s_out, tclr_out, L_out,
                       (hipStream_t)stream);
    if (er == hipSuccess) er = launch_sweep_count(kp, tclr_out, nshots, sweeps_out, (hipStream_t)stream);
  }
  if (er == hipSuccess && fail_out && !fused_fail)
    er = launch_failure(code->dev, e0, z_out, nshots, fail_out, (hipStream_t)stream);
  return er == hipSuccess ? LAIM_OK : hip_fail(er, "decode kernels");
}

}  // namespace laim

extern "C" {

laim_status laim_decode_rounds(const laim_code* code, const laim_decode_params* params,
                               const uint8_t* e0, uint64_t shot0, int32_t nshots, void* workspace,
                               size_t ws_bytes, uint8_t* z_out, uint8_t* s_out, int32_t* tclr_out,
                               float* L_out, int32_t* sweeps_out, uint8_t* fail_out, int32_t form,
                               laim_stream stream) {
  return decode_common(code, params, e0, shot0, nshots, workspace, ws_bytes, z_out, s_out, tclr_out,
                       L_out, sweeps_out, fail_out, form, nullptr, stream);
}

laim_status laim_decode_rounds_cfg(const laim_code* code, const laim_decode_params* params,
                                   const uint8_t* e0, uint64_t shot0, int32_t nshots,
                                   void* workspace, size_t ws_bytes, uint8_t* z_out, uint8_t* s_out,
                                   int32_t* tclr_out, float* L_out, int32_t* sweeps_out,
                                   uint8_t* fail_out, const laim_resident_cfg* cfg,
                                   laim_stream stream) {
  if (!cfg) {
    set_error("cfg is NULL");
    return LAIM_EINVAL;
  }
  return decode_common(code, params, e0, shot0, nshots, workspace, ws_bytes, z_out, s_out, tclr_out,
                       L_out, sweeps_out, fail_out, LAIM_FORM_RESIDENT, cfg, stream);
}

laim_status laim_decode_continuous(const laim_code* code, const laim_continuous_params* params,
                                   const uint8_t* e0, uint64_t shot0, int32_t nshots,
                                   void* workspace, size_t ws_bytes, uint8_t* z_out, uint8_t* s_out,
                                   double* tclr_out, int32_t* counts_out, int32_t* steps_out,
                                   uint8_t* fail_out, int32_t checks_per_thread, laim_stream stream) {
  if (!code || !params || nshots < 0 || (nshots > 0 && (!e0 || !z_out || !s_out || !tclr_out))) {
    set_error("laim_decode_continuous: bad arguments");
    return LAIM_EINVAL;
  }
  const laim_continuous_params& p = *params;
  if (p.bp != 0 && p.bp != 1) {
    set_error("bp must be 0 (min-sum) or 1 (sum-product)");
    return LAIM_EINVAL;
  }
  if (!(p.q > 0.0 && p.q < 1.0) || !(p.clamp > 0.0f) || !(p.alpha > 0.0f)) {
    set_error("q must lie in (0, 1); clamp and alpha must be positive");
    return LAIM_EINVAL;
  }
  if (!(p.dt > 0.0) || !(p.tau > 0.0) || !(p.t_max >= 0.0) || !(p.t_max / p.dt <= 2147483647.0)) {
    set_error("dt and tau must be positive and 0 <= t_max / dt <= 2^31 - 1");
    return LAIM_EINVAL;
  }
  if (checks_per_thread != 0 && checks_per_thread != 1 && checks_per_thread != 2 &&
      checks_per_thread != 4 && checks_per_thread != 8) {
    set_error("checks_per_thread must be 0, 1, 2, 4 or 8");
    return LAIM_EINVAL;
  }
  if (nshots == 0) return LAIM_OK;
  if (!workspace || ws_bytes < LAIM_CONTINUOUS_WORKSPACE_BYTES || ((uintptr_t)workspace) % 256) {
    set_error("a 256-byte aligned workspace of %d bytes is needed", LAIM_CONTINUOUS_WORKSPACE_BYTES);
    return LAIM_ENOMEM;
  }
  if (fail_out && code->dev.kw > 64) {
    set_error("more than 2048 logicals are not supported");
    return LAIM_EUNSUP;
  }
  CtmParamsDev P;
  P.bp = p.bp;
  P.alpha = p.alpha;
  P.pi = (float)log(p.q / (1.0 - p.q));
  P.clamp = p.clamp;
  P.lam = (float)(p.dt / p.tau);
  P.dt = p.dt;
  P.max_steps = (int32_t)floor(p.t_max / p.dt + 0.5);
  P.evidence = p.evidence ? 1 : 0;
  P.seed = p.seed;
  P.skip = p.skip_fixed ? 1 : 0;
  CtmShape sh;
  if (!ctm_shape(code->dev, P, checks_per_thread, code->device, &sh)) return LAIM_EUNSUP;
  DeviceGuard g(code->device);
  hipError_t er = launch_ctm(code->dev, P, sh, e0, shot0, nshots, workspace, z_out, s_out, tclr_out,
                             counts_out, steps_out, fail_out, (hipStream_t)stream);
  return er == hipSuccess ? LAIM_OK : hip_fail(er, "continuous-machine kernel");
}

// Whether H is a chain over bits 0..n-1 in index order: each check is {v, v + 1}
// for one v < n - 1, or {0, n - 1} when periodic (m = n), and each appears once.
// swap0: bit 0 sums its right check's message first (its left check has the
// larger index); a chain where another bit does so is not taken.
static bool bit_chain(const laim_code* code, bool* periodic, int32_t* swap0) {
  const int32_t n = code->n, m = code->m;
  if (m != n - 1 && m != n) return false;
  const bool per = (m == n);
  if (n < (per ? 3 : 2)) return false;
  std::vector<int32_t> left((size_t)n, -1), right((size_t)n, -1);
  for (int32_t c = 0; c < m; ++c) {
    const int32_t b0 = code->h_rowptr[c];
    if (code->h_rowptr[c + 1] - b0 != 2) return false;
    int32_t a = code->h_col[b0], b = code->h_col[b0 + 1];
    if (a > b) std::swap(a, b);
    if (b == a + 1) {
      if (right[a] >= 0 || left[b] >= 0) return false;
      right[a] = left[b] = c;
    } else if (per && a == 0 && b == n - 1) {
      if (left[0] >= 0 || right[n - 1] >= 0) return false;
      left[0] = right[n - 1] = c;
    } else {
      return false;
    }
  }
  *swap0 = 0;
  for (int32_t v = 0; v < n; ++v)
    if (left[v] >= 0 && right[v] >= 0 && left[v] > right[v]) {
      if (v != 0) return false;
      *swap0 = 1;
    }
  *periodic = per;
  return true;
}

laim_status laim_decode_bitcentric_form(const laim_code* code, double q, const uint8_t* e0,
                                        int32_t nshots, int32_t iters, int32_t form, uint8_t* z_out,
                                        int32_t* iclr_out, double* L_out, laim_stream stream) {
  if (!code || nshots < 0 || iters < 0 || !(q > 0.0 && q < 1.0) ||
      (form != LAIM_BC_AUTO && form != LAIM_BC_CHAIN && form != LAIM_BC_BLOCK) ||
      (nshots > 0 && (!e0 || !z_out || !iclr_out))) {
    set_error("laim_decode_bitcentric: bad arguments");
    return LAIM_EINVAL;
  }
  for (int32_t c = 0; c < code->m; ++c)
    if (code->h_rowptr[c + 1] - code->h_rowptr[c] != 2) {
      set_error("the bit-centric machine needs every check of degree 2");
      return LAIM_EUNSUP;
    }
  bool periodic = false;
  int32_t swap0 = 0, K = 0, nl = 0, S = 0;
  // on a cycle some bit has its left check at the larger index; the chain
  // form takes the cycles where that bit is bit 0 (and only bit 0)
  const bool chain = form != LAIM_BC_BLOCK && bit_chain(code, &periodic, &swap0) &&
                     swap0 == (periodic ? 1 : 0) && bitchain_shape(code->n, periodic, &K, &nl, &S);
  if (form == LAIM_BC_CHAIN && !chain) {
    set_error("the chain form needs a chain of 2..1008 bits (3..1024 periodic) whose bits "
              "other than bit 0 list their left check first");
    return LAIM_EUNSUP;
  }
  if (nshots == 0) return LAIM_OK;
  int32_t nt = 0;
  size_t lds = 0;
  if (!chain && !bitcentric_shape(code->dev, code->device, &nt, &lds)) return LAIM_EUNSUP;
  DeviceGuard g(code->device);
  hipError_t er = chain ? launch_bitchain(code->n, periodic, K, nl, S, q, e0, nshots, iters, z_out,
                                          iclr_out, L_out, (hipStream_t)stream)
                        : launch_bitcentric(code->dev, q, e0, nshots, iters, nt, lds, z_out,
                                            iclr_out, L_out, (hipStream_t)stream);
  return er == hipSuccess ? LAIM_OK : hip_fail(er, "bit-centric kernel");
}

laim_status laim_decode_bitcentric(const laim_code* code, double q, const uint8_t* e0,
                                   int32_t nshots, int32_t iters, uint8_t* z_out, int32_t* iclr_out,
                                   double* L_out, laim_stream stream) {
  return laim_decode_bitcentric_form(code, q, e0, nshots, iters, LAIM_BC_AUTO, z_out, iclr_out,
                                     L_out, stream);
}

laim_status laim_set_resident_cfg(laim_code* code, int32_t bp, const laim_resident_cfg* cfg) {
  if (!code || (bp != 0 && bp != 1)) {
    set_error("laim_set_resident_cfg: bad arguments");
    return LAIM_EINVAL;
  }
  if (!cfg) {
    code->has_cfg[bp] = false;
    return LAIM_OK;
  }
  ResidentShape sh;
  if (!resident_shape(code->dev, bp, cfg, &sh, code->device)) return LAIM_EINVAL;
  code->cfg[bp] = *cfg;
  code->has_cfg[bp] = true;
  return LAIM_OK;
}

laim_status laim_get_resident_cfg(const laim_code* code, int32_t bp, laim_resident_cfg* cfg) {
  if (!code || !cfg || (bp != 0 && bp != 1)) {
    set_error("laim_get_resident_cfg: bad arguments");
    return LAIM_EINVAL;
  }
  ResidentShape sh;
  if (!resident_shape(code->dev, bp, code->has_cfg[bp] ? &code->cfg[bp] : nullptr, &sh,
                      code->device))
    return LAIM_EUNSUP;
  cfg->threads_per_shot = sh.nt;
  cfg->checks_per_thread = sh.cpt;
  cfg->shots_per_block = sh.spb;
  return LAIM_OK;
}

}  // extern "C"
