// Host planner: validation, constraint classes, evaluation kinds, inverse-DFT
// weights, length-bucketed segments and the device image.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <tuple>

namespace pcls {

static thread_local std::string g_error;

int32_t set_error(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

void clear_error() { g_error.clear(); }

const char* last_error() { return g_error.c_str(); }

// Whether a symmetric constraint holds with exactly t of its k literals true
// (paper: Table 2 and Appendix A).
static bool holds(int type, int k, int param, int t) {
  switch (type) {
    case PCLS_OR: return t >= 1;
    case PCLS_XOR: return (t & 1) == param;
    case PCLS_CARD_GE: return t >= param;
    case PCLS_NAE: return t > 0 && t < k;
    case PCLS_EO: return t == 1;
    case PCLS_AMO: return t <= 1;
    case PCLS_EK: return t == param;
  }
  return false;
}

struct ClassKey {
  int type, k, param;
  bool operator<(const ClassKey& o) const {
    return std::tie(type, k, param) < std::tie(o.type, o.k, o.param);
  }
};

// Evaluation kind from the shape of the spectrum.  FE = sum_t sp_t Pr[T = t]
// where Pr[T = 0] = prod u_i, Pr[T = k] = prod p_i (u = (1+y)/2, p = (1-y)/2)
// and sum_t (-1)^t Pr[T = t] = prod y_i.
static int pmf_window(const std::vector<int>& sp, float* d, float* h, int nd);

// LDS bank-aware order of one run of short constraints (one lane per pair).
// A wave instruction reads slot j of a block of consecutive constraints; with T
// restarts per tile the rows of its variables occupy bank groups v mod (64/T')
// for blocks of 64/T' constraints (T' = T, or T/2 with two restarts per lane),
// and variables in the same group serialise.  For each position (relative to
// the segment start, so blocks align with the kernel's chunks) the greedy picks,
// among the next 16 constraints of the run and their cyclic slot rotations,
// the one adding the fewest same-group pairs over the (block, groups) layouts
// (64, 64), (64, 32), (32, 16) and (16, 8).  Symmetric constraints do not depend
// on their literal order, so rotating the slots changes no value.
static void bank_aware_order(const int32_t* row_ptr, const int32_t* lit, int k, int32_t* run, int len, int seg_off,
                             std::vector<uint8_t>& rot_of) {
  constexpr int kWindow = 16, kCfg = 4;
  const int blk[kCfg] = {64, 64, 32, 16}, mask[kCfg] = {63, 31, 15, 7};
  uint16_t occ[kCfg][8][64];
  struct Cand {
    int32_t c;
    uint8_t res[8];  // variable mod 64 per slot
  };
  auto make = [&](int32_t c) {
    Cand d{c, {}};
    for (int i = 0; i < k; ++i) {
      const int l = lit[row_ptr[c] + i];
      d.res[i] = (uint8_t)(((l > 0 ? l : -l) - 1) & 63);
    }
    return d;
  };
  // window: the first kWindow not-yet-placed constraints of the run, in run order
  Cand win[kWindow];
  int nwin = 0, next = 0;
  while (nwin < kWindow && next < len) win[nwin++] = make(run[next++]);
  std::vector<int32_t> out;
  out.reserve(len);
  for (int q = 0; q < len; ++q) {
    const int pos = seg_off + q;
    for (int c = 0; c < kCfg; ++c)
      if (pos % blk[c] == 0) std::memset(occ[c], 0, sizeof occ[c]);
    int best = 0, best_rot = 0, best_cost = 1 << 30;
    for (int w = 0; w < nwin && best_cost > 0; ++w) {
      for (int r = 0; r < k && best_cost > 0; ++r) {
        int cost = 0;
        for (int j = 0; j < k; ++j) {
          const int v = win[w].res[(j + r) % k];
          for (int c = 0; c < kCfg; ++c) cost += occ[c][j][v & mask[c]];
        }
        if (cost < best_cost) {
          best_cost = cost;
          best = w;
          best_rot = r;
        }
      }
    }
    const Cand chosen = win[best];
    for (int j = 0; j < k; ++j) {
      const int v = chosen.res[(j + best_rot) % k];
      for (int c = 0; c < kCfg; ++c) ++occ[c][j][v & mask[c]];
    }
    rot_of[(size_t)chosen.c] = (uint8_t)best_rot;
    out.push_back(chosen.c);
    for (int w = best; w + 1 < nwin; ++w) win[w] = win[w + 1];  // keep run order
    --nwin;
    if (next < len) win[nwin++] = make(run[next++]);
  }
  std::copy(out.begin(), out.end(), run);
}

// LDS bank balance of the long buckets.  One wave instruction of the
// long-constraint kernels reads slot lig*J + j (J = kmax/G) of every lane group
// of a chunk; with one restart per tile that is the 64/G constraints of the
// chunk on G lanes each, and x of variable v (and its gradient accumulator)
// sits in LDS bank v mod 64.  A symmetric constraint's literals and pad slots
// may take any of its slots, so moving one between instructions j1 != j2 of
// its own constraint changes no value.  A local search swaps slot pairs of one
// constraint while that lowers the sum over the chunk's instructions of the
// squared bank counts (two passes over each constraint's slot pairs: planning
// work O(L kmax), so the search stops at the 64 bucket; from 96 literals a
// chunk holds at most 4 constraints and the gathers are few per literal).
// seg: the segment's transposed codes [slot][c_count].
static void balance_long_slots(int32_t* seg, int c_count, int kmax, int G) {
  const int J = kmax / G, chunk = 64 / G;
  std::vector<int> cnt((size_t)J * 64);
  auto bank = [](int32_t code) { return (int)((uint32_t)code & 0x7fffffffu) & 63; };
  for (int c0 = 0; c0 < c_count; c0 += chunk) {
    const int c1 = std::min(c_count, c0 + chunk);
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int q = c0; q < c1; ++q)
      for (int s = 0; s < kmax; ++s) ++cnt[(size_t)(s % J) * 64 + bank(seg[(size_t)s * c_count + q])];
    for (int pass = 0; pass < 2; ++pass) {
      bool changed = false;
      for (int q = c0; q < c1; ++q) {
        for (int s1 = 0; s1 < kmax; ++s1) {
          for (int s2 = s1 + 1; s2 < kmax; ++s2) {
            const int j1 = s1 % J, j2 = s2 % J;
            if (j1 == j2) continue;
            int32_t& a = seg[(size_t)s1 * c_count + q];
            int32_t& b = seg[(size_t)s2 * c_count + q];
            const int b1 = bank(a), b2 = bank(b);
            if (b1 == b2) continue;
            // a moves j1 -> j2, b moves j2 -> j1: change of the sum of squares
            const int d = 2 * (cnt[(size_t)j2 * 64 + b1] - cnt[(size_t)j1 * 64 + b1] + 1) +
                          2 * (cnt[(size_t)j1 * 64 + b2] - cnt[(size_t)j2 * 64 + b2] + 1);
            if (d < 0) {
              --cnt[(size_t)j1 * 64 + b1];
              ++cnt[(size_t)j2 * 64 + b1];
              --cnt[(size_t)j2 * 64 + b2];
              ++cnt[(size_t)j1 * 64 + b2];
              std::swap(a, b);
              changed = true;
            }
          }
        }
      }
      if (!changed) break;
    }
  }
}

static void classify(const std::vector<int>& sp, bool force_generic, int table, ClassRec& C) {
  const int k = (int)sp.size() - 1;
  bool all_eq = true, tail_eq = true, head_eq = true, alt = true, mid_eq = true;
  for (int t = 0; t <= k; ++t) {
    if (sp[t] != sp[0]) all_eq = false;
    if (t >= 1 && sp[t] != sp[1]) tail_eq = false;
    if (t <= k - 1 && sp[t] != sp[0]) head_eq = false;
    if (sp[t] != ((t & 1) ? -sp[0] : sp[0])) alt = false;
    if (t >= 1 && t <= k - 1 && sp[t] != sp[1]) mid_eq = false;
  }
  C.a = C.b = C.c1 = C.c2 = C.c0 = 0.f;
  if (all_eq) {
    C.kind = KIND_CONST;
    C.c0 = (float)sp[0];
    return;
  }
  if (!force_generic) {
    if (tail_eq) {  // FE = sp_1 + (sp_0 - sp_1) prod u
      C.kind = KIND_PROD1;
      C.a = 0.5f;
      C.b = 0.5f;
      C.c0 = (float)sp[1];
      C.c1 = (float)(sp[0] - sp[1]);
      return;
    }
    if (head_eq) {  // FE = sp_0 + (sp_k - sp_0) prod p
      C.kind = KIND_PROD1;
      C.a = 0.5f;
      C.b = -0.5f;
      C.c0 = (float)sp[0];
      C.c1 = (float)(sp[k] - sp[0]);
      return;
    }
    if (alt) {  // FE = sp_0 prod y
      C.kind = KIND_PROD1;
      C.a = 0.f;
      C.b = 1.f;
      C.c0 = 0.f;
      C.c1 = (float)sp[0];
      return;
    }
    if (k >= 3 && mid_eq) {  // FE = s + (sp_0 - s) prod u + (sp_k - s) prod p
      C.kind = KIND_PROD2;
      C.a = 0.5f;
      C.b = 0.5f;
      C.c0 = (float)sp[1];
      C.c1 = (float)(sp[0] - sp[1]);
      C.c2 = (float)(sp[k] - sp[1]);
      return;
    }
    const int w = pmf_window(sp, nullptr, nullptr, 0);
    const int kb = kBucketKmax[bucket_of(k, table)];
    if ((k <= kPmfMaxK && w <= kPmfWindow) || (k > kPmfMaxK && kb <= kPmfGroupMaxK && 2 * w <= kb)) {
      C.kind = KIND_PMF;
      return;
    }
  }
  C.kind = KIND_DFT;
}

// PMF kind: the shorter of the two windows.  Counting true literals,
// FE = sp_k + sum_{t < w} (sp_t - sp_k) Pr[T = t] with w = 1 + the last t where
// sp_t != sp_k; counting false ones (F = k - T), FE = sp_0 + sum_{f < w}
// (sp_{k-f} - sp_0) Pr[F = f].  Returns w; fills d[0..nd-1] (zero past w) and h.
static int pmf_window(const std::vector<int>& sp, float* d, float* h, int nd = kPmfWindow) {
  const int k = (int)sp.size() - 1;
  int wt = 0, wf = 0;
  for (int t = 0; t <= k; ++t)
    if (sp[t] != sp[k]) wt = t + 1;
  for (int f = 0; f <= k; ++f)
    if (sp[k - f] != sp[0]) wf = f + 1;
  const bool count_true = wt <= wf;
  const int w = count_true ? wt : wf;
  if (d) {
    for (int c = 0; c < nd; ++c)
      d[c] = (c < w && c <= k) ? (float)(count_true ? sp[c] - sp[k] : sp[k - c] - sp[0]) : 0.f;
    *h = count_true ? 0.5f : -0.5f;
  }
  return w;
}

// Whether a long PMF class counts false literals (h = -1/2 in its record).
static bool pmf_counts_false_of(const std::vector<NodeRec>& nodes, const ClassRec& C) {
  float rec[40];
  std::memcpy(rec, &nodes[(size_t)C.node_off], sizeof rec);
  return rec[32] < 0.f;
}

// Inverse-DFT weights over the K = k + 1 roots of unity.  With
// Q_m = prod_i (alpha_m + beta_m y_i), alpha_m = (1 + w^m)/2, beta_m = (1 - w^m)/2,
// w = exp(2 pi i / K), Q_m is the characteristic function of T at 2 pi m / K,
// so Pr[T = t] = (1/K) sum_m Q_m w^-tm and FE = sum_m chat_m Q_m with
// chat_m = (1/K) sum_t sp_t w^-tm.  The angles use exact integer reduction
// (t m mod K) and FP64 arithmetic; results are rounded once to float32.
static void dft_weights(const std::vector<int>& sp, ClassRec& C, std::vector<NodeRec>& nodes) {
  const int k = (int)sp.size() - 1;
  const int K = k + 1;
  const double two_pi = 6.283185307179586476925286766559;
  auto chat = [&](int m, double& re, double& im) {
    re = im = 0.0;
    for (int t = 0; t <= k; ++t) {
      long r = ((long)t * m) % K;
      double ang = two_pi * (double)r / (double)K;
      re += sp[t] * std::cos(ang);
      im -= sp[t] * std::sin(ang);
    }
    re /= K;
    im /= K;
  };
  double c0r, c0i;
  chat(0, c0r, c0i);
  C.c0 = (float)c0r;
  C.nyquist = (K % 2 == 0) ? 1 : 0;
  C.n_nodes = (K - 1) / 2;  // complex nodes 1..(K-1)/2; K even adds the real node K/2
  C.node_off = (int32_t)nodes.size();
  for (int m = 1; m <= C.n_nodes; ++m) {
    double wr, wi;
    chat(m, wr, wi);
    double ang = two_pi * (double)m / (double)K;
    double er = std::cos(ang), ei = std::sin(ang);
    // alpha + beta = 1 exactly in float32 (the larger real part is rounded, the
    // other is 1 minus it, exact by Sterbenz), so a pad slot (y = 1) has the
    // factor 1 + 0i exactly
    float far = (float)(0.5 * (1.0 + er)), fbr = (float)(0.5 * (1.0 - er));
    if (far >= 0.5f)
      fbr = 1.0f - far;
    else
      far = 1.0f - fbr;
    const float fai = (float)(0.5 * ei);
    const double ar = far, br = fbr, ai = fai, bi = -(double)fai;
    NodeRec nd;
    nd.ar = far;
    nd.ai = fai;
    nd.br = fbr;
    nd.bi = -fai;
    nd.wr = (float)(2.0 * wr);
    nd.wi = (float)(2.0 * wi);
    nd.gr = (float)(2.0 * (wr * br - wi * bi));
    nd.gi = (float)(2.0 * (wr * bi + wi * br));
    nodes.push_back(nd);
  }
  if (C.nyquist) {
    double s = 0.0;
    for (int t = 0; t <= k; ++t) s += (t & 1) ? -sp[t] : sp[t];
    C.c1 = (float)(s / K);
  }
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int32_t build_plan(int32_t n, int32_t m, const int32_t* row_ptr, const int32_t* lit, const int8_t* type,
                   const int32_t* param, const float* weight, const pcls_plan_options* options,
                   pcls_problem** out, size_t* workspace_bytes) {
  if (!out || !workspace_bytes) return set_error(PCLS_E_INVALID, "out and workspace_bytes must not be NULL");
  *out = nullptr;
  *workspace_bytes = 0;
  if (n < 1) return set_error(PCLS_E_INVALID, "n_vars must be >= 1 (got %d)", n);
  if (n > (1 << 29)) return set_error(PCLS_E_UNSUPPORTED, "n_vars %d exceeds 2^29", n);
  if (m < 0) return set_error(PCLS_E_INVALID, "n_cons must be >= 0 (got %d)", m);
  if (!row_ptr) return set_error(PCLS_E_INVALID, "row_ptr must not be NULL");
  if (m > 0 && !type) return set_error(PCLS_E_INVALID, "type must not be NULL");
  if (row_ptr[0] != 0) return set_error(PCLS_E_INVALID, "row_ptr[0] must be 0 (got %d)", row_ptr[0]);
  for (int c = 0; c < m; ++c) {
    int k = row_ptr[c + 1] - row_ptr[c];
    if (k < 1) return set_error(PCLS_E_INVALID, "constraint %d has length %d (row_ptr must increase)", c, k);
    if (k > kMaxK) return set_error(PCLS_E_UNSUPPORTED, "constraint %d has %d literals (max %d)", c, k, kMaxK);
  }
  const int64_t L = row_ptr[m];
  if (L > 0 && !lit) return set_error(PCLS_E_INVALID, "lit must not be NULL");
  const bool force_generic = options && options->force_generic;
  const int acc_bits = options ? options->accumulator_bits : 0;
  if (acc_bits != 0 && acc_bits != 32 && acc_bits != 64)
    return set_error(PCLS_E_INVALID, "accumulator_bits must be 0, 32 or 64 (got %d)", acc_bits);
  const int table = options ? options->bucket_table : 0;
  if (table < 0 || table >= kNumBucketTables)
    return set_error(PCLS_E_INVALID, "bucket_table must be 0 or 1 (got %d)", table);

  std::vector<int32_t> stamp((size_t)n, -1);
  for (int c = 0; c < m; ++c) {
    int ty = type[c];
    int k = row_ptr[c + 1] - row_ptr[c];
    int pr = param ? param[c] : 0;
    if (ty < PCLS_OR || ty > PCLS_EK) return set_error(PCLS_E_INVALID, "constraint %d: unknown type %d", c, ty);
    if (ty == PCLS_XOR && (pr < 0 || pr > 1))
      return set_error(PCLS_E_INVALID, "constraint %d: XOR parity must be 0 or 1 (got %d)", c, pr);
    if ((ty == PCLS_CARD_GE || ty == PCLS_EK) && (pr < 0 || pr > k))
      return set_error(PCLS_E_INVALID, "constraint %d: kappa %d outside [0, %d]", c, pr, k);
    if (weight && !std::isfinite(weight[c]))
      return set_error(PCLS_E_INVALID, "constraint %d: weight is not finite", c);
    for (int i = row_ptr[c]; i < row_ptr[c + 1]; ++i) {
      int l = lit[i];
      if (l == 0 || l == INT32_MIN || (l > 0 ? l : -l) > n)
        return set_error(PCLS_E_INVALID, "constraint %d: literal %d out of range [1, %d]", c, l, n);
      int v = l > 0 ? l : -l;
      if (stamp[v - 1] == c)
        return set_error(PCLS_E_DUPVAR, "constraint %d: variable %d occurs twice", c, v);
      stamp[v - 1] = c;
    }
  }

  pcls_problem* P = new (std::nothrow) pcls_problem();
  if (!P) return set_error(PCLS_E_INVALID, "out of host memory");
  P->n = n;
  P->m = m;
  P->L = L;
  P->force_generic = force_generic ? 1 : 0;
  P->bucket_table = table;

  // ---- classes
  std::map<ClassKey, int> class_of;
  std::vector<int> cls_orig((size_t)m);
  double f_const = 0.0;
  for (int c = 0; c < m; ++c) {
    int ty = type[c];
    int k = row_ptr[c + 1] - row_ptr[c];
    int pr = (ty == PCLS_XOR || ty == PCLS_CARD_GE || ty == PCLS_EK) ? (param ? param[c] : 0) : 0;
    ClassKey key{ty, k, pr};
    auto it = class_of.find(key);
    if (it == class_of.end()) {
      std::vector<int> sp((size_t)k + 1);
      for (int t = 0; t <= k; ++t) sp[t] = holds(ty, k, pr, t) ? -1 : 1;
      ClassRec C{};
      C.k = k;
      classify(sp, force_generic, P->bucket_table, C);
      if (C.kind == KIND_DFT) dft_weights(sp, C, P->nodes);
      if (C.kind == KIND_PMF && k <= kPmfMaxK) {
        NodeRec N{};
        float d[kPmfWindow], h;
        C.nyquist = pmf_window(sp, d, &h, kPmfWindow);  // PMF: the window w (counts kept)
        N.ar = d[0];
        N.ai = d[1];
        N.br = d[2];
        N.bi = d[3];
        N.wr = h;
        C.c0 = (float)(h > 0.f ? sp[k] : sp[0]);
        C.node_off = (int32_t)P->nodes.size();
        C.n_nodes = 1;
        P->nodes.push_back(N);
      } else if (C.kind == KIND_PMF) {
        // lane-group PMF: d_0..d_31, h, threshold flag, in five node records
        float rec[40] = {};
        float h;
        const int w = pmf_window(sp, rec, &h, 32);
        C.nyquist = w;
        rec[32] = h;
        bool thr = true;  // d constant on the window
        for (int c = 1; c < w; ++c)
          if (rec[c] != rec[0]) thr = false;
        rec[33] = thr ? 1.f : 0.f;
        C.c0 = (float)(h > 0.f ? sp[k] : sp[0]);
        C.node_off = (int32_t)P->nodes.size();
        C.n_nodes = 5;
        for (int r = 0; r < 5; ++r) {
          NodeRec N;
          std::memcpy(&N, rec + 8 * r, sizeof N);
          P->nodes.push_back(N);
        }
      }
      C.sp_off = (int32_t)P->sp.size();
      for (int t = 0; t <= k; ++t) P->sp.push_back((int8_t)sp[t]);
      int id = (int)P->classes.size();
      P->classes.push_back(C);
      it = class_of.emplace(key, id).first;
    }
    cls_orig[c] = it->second;
    const float w = weight ? weight[c] : 1.0f;
    if (w != 1.0f) P->unit_weights = 0;
    f_const += (double)w * (double)P->classes[it->second].c0;
    P->max_k = std::max(P->max_k, k);
  }
  P->f_const = (float)f_const;
  P->acc_bits = acc_bits;

  // ---- fixed-point scales (see plan.h)
  {
    std::vector<double> occ((size_t)n, 0.0);
    P->occ.assign((size_t)n, 0);
    for (int c = 0; c < m; ++c) {
      const double w = std::fabs(weight ? (double)weight[c] : 1.0);
      if (P->classes[cls_orig[c]].kind == KIND_CONST) continue;
      P->max_w = std::max(P->max_w, w);
      P->maxsum_f += w;
      for (int i = row_ptr[c]; i < row_ptr[c + 1]; ++i) {
        const int l = lit[i];
        occ[(size_t)((l > 0 ? l : -l) - 1)] += w;
        P->occ[(size_t)((l > 0 ? l : -l) - 1)] += 1;
      }
    }
    for (double v : occ) P->maxsum_g = std::max(P->maxsum_g, v);
    auto clog2 = [](double x) { return (int)std::ceil(std::log2(x)); };
    const double margin = 1.01;  // FP32 rounding of a term bounded by 1 in exact arithmetic
    const int lg = clog2(P->maxsum_g * margin + 1.0), lw = clog2(P->max_w * margin + 1.0);
    // 64-bit: a term times 2^S must stay below 2^50 (rounding through the FP64
    // significand) and a sum below 2^61; 32-bit: below 2^29 and 2^30.
    P->s_g64 = std::min(61 - lg, 50 - lw);
    P->s_g32 = std::min(30 - lg, 29 - lw);
    P->s_f = 50 - clog2(P->maxsum_f * margin + 1.0);
    if (P->s_g64 < 8 || P->s_f < 8) {
      int32_t st = set_error(PCLS_E_UNSUPPORTED, "constraint weights too large for fixed-point accumulation");
      delete P;
      return st;
    }
    if (acc_bits == 32 && P->s_g32 < 8) {
      int32_t st = set_error(PCLS_E_UNSUPPORTED, "weights or degrees too large for a 32-bit gradient accumulator");
      delete P;
      return st;
    }
  }

  // ---- planned order: (kind, bucket, class, original index); CONST last
  std::vector<int32_t> order((size_t)m);
  for (int c = 0; c < m; ++c) order[c] = c;
  auto seg_key = [&](int c) {
    const ClassRec& C = P->classes[cls_orig[c]];
    int kind = C.kind;
    int b = kind == KIND_CONST ? 0 : bucket_of(C.k, P->bucket_table);
    return std::make_tuple(kind, b, cls_orig[c], c);
  };
  std::sort(order.begin(), order.end(), [&](int a, int b) { return seg_key(a) < seg_key(b); });
  // bank-aware order inside each class run of the short buckets (one lane per pair)
  std::vector<uint8_t> rot_of((size_t)m, 0);
  {
    int seg_start = 0;
    for (int a = 0; a < m;) {
      const ClassRec& C = P->classes[cls_orig[order[a]]];
      if (C.kind == KIND_CONST) break;
      const int b = bucket_of(C.k, P->bucket_table);
      if (a > 0) {
        const ClassRec& Cp = P->classes[cls_orig[order[a - 1]]];
        if (Cp.kind != C.kind || bucket_of(Cp.k, P->bucket_table) != b) seg_start = a;
      }
      int e = a;
      while (e < m && cls_orig[order[e]] == cls_orig[order[a]]) ++e;
      if (kBucketKmax[b] <= 8 && group_size(C.kind, kBucketKmax[b]) == 1)
        bank_aware_order(row_ptr, lit, C.k, order.data() + a, e - a, a - seg_start, rot_of);
      a = e;
    }
  }
  P->perm = order;
  P->c_k.resize(m);
  P->c_cls.resize(m);
  P->c_w.resize(m);
  P->row_ptr.resize((size_t)m + 1);
  P->lit.resize((size_t)L);
  P->row_ptr[0] = 0;
  for (int j = 0; j < m; ++j) {
    int c = order[j];
    int k = row_ptr[c + 1] - row_ptr[c];
    P->c_k[j] = k;
    P->c_cls[j] = cls_orig[c];
    P->c_w[j] = weight ? weight[c] : 1.0f;
    P->row_ptr[j + 1] = P->row_ptr[j] + k;
    for (int i = 0; i < k; ++i) {
      int l = lit[row_ptr[c] + (i + rot_of[(size_t)c]) % k];
      int v = (l > 0 ? l : -l) - 1;
      P->lit[P->row_ptr[j] + i] = (v << 1) | (l < 0 ? 1 : 0);
    }
  }

  // ---- segments and their transposed literal blocks
  int j = 0;
  while (j < m) {
    const ClassRec& C0 = P->classes[P->c_cls[j]];
    if (C0.kind == KIND_CONST) break;
    int b = bucket_of(C0.k, P->bucket_table);
    int e = j;
    Segment S{};
    S.kind = C0.kind;
    S.bucket = b;
    S.c_begin = j;
    S.k_fixed = C0.k;
    S.cls_fixed = P->c_cls[j];
    S.m_max = 0;
    while (e < m) {
      const ClassRec& C = P->classes[P->c_cls[e]];
      if (C.kind != S.kind || bucket_of(C.k, P->bucket_table) != b) break;
      if (C.k != S.k_fixed) S.k_fixed = 0;
      if (P->c_cls[e] != S.cls_fixed) S.cls_fixed = -1;
      if (C.kind == KIND_DFT) S.m_max = std::max(S.m_max, C.n_nodes);
      if (C.kind == KIND_PMF) S.m_max = std::max(S.m_max, C.nyquist);
      ++e;
    }
    S.c_count = e - j;
    const int kmax = kBucketKmax[b];
    S.lit_base = (int32_t)P->litT.size();
    P->litT.resize(P->litT.size() + (size_t)kmax * S.c_count, -1);
    for (int q = 0; q < S.c_count; ++q) {
      int cj = j + q;
      for (int i = 0; i < P->c_k[cj]; ++i) {
        // kernel code: variable in the low bits, sign in bit 31 (flipped onto x and
        // onto the gradient term with one XOR each)
        const uint32_t code = (uint32_t)P->lit[P->row_ptr[cj] + i];
        P->litT[(size_t)S.lit_base + (size_t)i * S.c_count + q] = (int32_t)((code >> 1) | ((code & 1u) << 31));
      }
      // slots past the constraint's length code a pad row (x = +1) with the sign
      // that makes the slot's factor exactly 1: y = -1 for the product node
      // (1 - y)/2 and for counts of false literals (h < 0), y = +1 otherwise
      const ClassRec& C = P->classes[P->c_cls[cj]];
      const bool neg = (C.kind == KIND_PROD1 && C.b < 0.f) || (C.kind == KIND_PMF && (C.k > kPmfMaxK && pmf_counts_false_of(P->nodes, C)));
      for (int i = P->c_k[cj]; i < kmax; ++i)
        P->litT[(size_t)S.lit_base + (size_t)i * S.c_count + q] =
            (int32_t)((uint32_t)(n + (q + i) % kPadRows) | (neg ? 0x80000000u : 0u));
    }
    const int G = group_size(S.kind, kmax);
    if (kmax > 8 && kmax <= 64) balance_long_slots(P->litT.data() + S.lit_base, S.c_count, kmax, G);
    P->max_group = std::max(P->max_group, G);
    P->max_bucket = std::max(P->max_bucket, b);
    P->segments.push_back(S);
    j = e;
  }
  P->n_pad = P->max_bucket > kMaxbShort ? kPadRows : 0;

  // ---- heaviest segments first (work per constraint), so that the light items
  // claimed last fill the gaps between waves
  std::stable_sort(P->segments.begin(), P->segments.end(), [](const Segment& a, const Segment& b) {
    auto cost = [](const Segment& s) {
      const int k = kBucketKmax[s.bucket];
      return s.kind == KIND_DFT ? 4 * k * (s.m_max + 1)
             : s.kind == KIND_PMF ? (k <= kPmfMaxK ? 6 * k : k * (k / 2 + 2))
             : (s.kind == KIND_PROD2 ? 2 * k : k);
    };
    return cost(a) > cost(b);
  });

  // ---- device image layout
  size_t off = 0;
  auto place = [&](size_t bytes) {
    off = align_up(off, 256);
    size_t at = off;
    off += bytes;
    return at;
  };
  P->off_segments = place(sizeof(Segment) * P->segments.size());
  P->off_classes = place(sizeof(ClassRec) * P->classes.size());
  P->off_nodes = place(sizeof(NodeRec) * P->nodes.size());
  P->off_sp = place(P->sp.size());
  P->off_litT = place(sizeof(int32_t) * P->litT.size());
  P->off_ck = place(sizeof(int32_t) * (size_t)m);
  P->off_ccls = place(sizeof(int32_t) * (size_t)m);
  P->off_cw = place(sizeof(float) * (size_t)m);
  P->off_rowptr = place(sizeof(int32_t) * ((size_t)m + 1));
  P->off_lit = place(sizeof(int32_t) * (size_t)L);
  P->off_occ = place(sizeof(int32_t) * (size_t)n);
  P->off_perm = place(sizeof(int32_t) * (size_t)m);
  size_t total = align_up(std::max<size_t>(off, 256), 256);
  P->image.assign(total, 0);
  auto put = [&](size_t at, const void* src, size_t bytes) {
    if (bytes) std::memcpy(P->image.data() + at, src, bytes);
  };
  put(P->off_segments, P->segments.data(), sizeof(Segment) * P->segments.size());
  put(P->off_classes, P->classes.data(), sizeof(ClassRec) * P->classes.size());
  put(P->off_nodes, P->nodes.data(), sizeof(NodeRec) * P->nodes.size());
  put(P->off_sp, P->sp.data(), P->sp.size());
  put(P->off_litT, P->litT.data(), sizeof(int32_t) * P->litT.size());
  put(P->off_ck, P->c_k.data(), sizeof(int32_t) * (size_t)m);
  put(P->off_ccls, P->c_cls.data(), sizeof(int32_t) * (size_t)m);
  put(P->off_cw, P->c_w.data(), sizeof(float) * (size_t)m);
  put(P->off_rowptr, P->row_ptr.data(), sizeof(int32_t) * ((size_t)m + 1));
  put(P->off_lit, P->lit.data(), sizeof(int32_t) * (size_t)L);
  put(P->off_occ, P->occ.data(), sizeof(int32_t) * (size_t)n);
  put(P->off_perm, P->perm.data(), sizeof(int32_t) * (size_t)m);

  *out = P;
  *workspace_bytes = total;
  clear_error();
  return PCLS_OK;
}

}  // namespace pcls
