// gfx950 kernels and C-ABI entry points of libpcls.
//
// Resident engine: one workgroup owns a tile of T restarts of one problem and
// keeps that tile's state x[n][T] and gradient g[n][T] in LDS for all steps of
// a launch.  Per step every constraint is evaluated for the T restarts
// (literal gather from LDS, node products, division-free prefix/suffix
// gradient, LDS atomic scatter), then x <- clip(x - lr g, -1, 1) in LDS.  HBM
// sees x once in and once out per launch plus the constraint stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "plan.h"

using namespace pcls;

namespace pcls {
const char* last_error();
}

namespace {

constexpr int kWave = 64;

// Read-only tables are read through the constant address space: a uniform
// address then becomes a scalar load instead of a vector load per lane.
template <class T>
using kptr = const __attribute__((address_space(4))) T*;
template <class T>
__device__ __forceinline__ kptr<T> kconst(const T* p) {
  return (kptr<T>)p;
}

struct cf {
  float r, i;
};

__device__ __forceinline__ cf cmul(cf a, cf b) {
  return {fmaf(a.r, b.r, -a.i * b.i), fmaf(a.r, b.i, a.i * b.r)};
}

template <int G>
struct Log2 {
  static constexpr int v = 1 + Log2<G / 2>::v;
};
template <>
struct Log2<1> {
  static constexpr int v = 0;
};

// Fixed-point accumulation of gradient and objective contributions in LDS.
// Integer LDS atomics run at the LDS's full rate whereas float LDS atomics are
// processed about one lane per few cycles; integer sums are also exact and
// independent of the order in which lanes arrive.  Contributions arrive
// pre-multiplied by 2^S (host-chosen so that no sum can overflow).
template <class AT>
struct FixedAcc;

template <>
struct FixedAcc<unsigned long long> {
  // |v| < 2^51: the FP64 sum 1.5 * 2^52 + v rounds v to the nearest integer,
  // and its bit pattern is kMagic + rint(v).  Gradient terms add the raw bit
  // patterns; a variable receives exactly one term per occurrence per step, so
  // value() removes count * kMagic once (all arithmetic mod 2^64 is exact).
  static constexpr unsigned long long kMagic = 0x4338000000000000ull;
  static __device__ __forceinline__ void add(unsigned long long* p, float v) {
    atomicAdd(p, (unsigned long long)__double_as_longlong((double)v + 6755399441055744.0));
  }
  static __device__ __forceinline__ float value(unsigned long long a, float inv, int count) {
    return (float)((double)(long long)(a - (unsigned long long)count * kMagic) * (double)inv);
  }
  // objective sums: integers with the magic already removed (fixed_term)
  static __device__ __forceinline__ float value_exact(unsigned long long a, float inv) {
    return (float)((double)(long long)a * (double)inv);
  }
};

template <>
struct FixedAcc<unsigned int> {
  // round to nearest (ties up) in one instruction: v_cvt_rpi computes floor(v + 1/2)
  static __device__ __forceinline__ void add(unsigned int* p, float v) {
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(v));
    atomicAdd(p, (unsigned int)r);
  }
  static __device__ __forceinline__ float value(unsigned int a, float inv, int) { return (float)(int)a * inv; }
};

// One objective term rounded to an integer (|v| < 2^51): per-lane sums of
// these are exact, so the objective does not depend on which lane took which
// constraint.
__device__ __forceinline__ long long fixed_term(float v) {
  return __double_as_longlong((double)v + 6755399441055744.0) - 0x4338000000000000LL;
}

// ---------------------------------------------------------------- lane groups
// A pair's G lanes sit at stride T inside the wave (lane = t + T * (lig + G * sub));
// with T = 1 and G <= 16 a group lies inside one 16-lane row, where DPP row
// operations reach its lanes (one VALU move, no LDS traffic).
template <int D>
__device__ __forceinline__ float row_shr(float v) {  // lane l reads lane l - D of its row
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 + D, 0xf, 0xf, true));
}
template <int D>
__device__ __forceinline__ float row_shl(float v) {  // lane l reads lane l + D of its row
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x100 + D, 0xf, 0xf, true));
}

// Leave-one-out product over a pair's G lanes: the product of the values of the
// other G - 1 lanes, by a butterfly of lane exchanges (log2 G levels; at level
// D a lane multiplies in the total of the block of D lanes at xor distance D,
// and both blocks' lanes form their union's total).  The exchanges reach the
// same partner lane at every tile width, so the result does not depend on T.
// With T = 1: distances 1 and 2 are DPP quad permutations, 4 two row shifts and
// a select, 8 a row rotation; 16 and every distance at T > 1 are wave shuffles.
template <int D>
__device__ __forceinline__ float grp_xchg(float v, int lig, int T) {
  if (T == 1) {
    if constexpr (D == 1) return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xf, 0xf, true));
    if constexpr (D == 2) return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xf, 0xf, true));
    if constexpr (D == 4) {
      const float up = row_shl<4>(v), dn = row_shr<4>(v);
      return (lig & 4) ? dn : up;
    }
    if constexpr (D == 8) return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xf, 0xf, true));
  }
  return __shfl_xor(v, D * T);
}

template <int G, int D = 1>
__device__ __forceinline__ void excl_levels(float& ex, float& tot, int lig, int T) {
  if constexpr (D < G) {
    const float o = grp_xchg<D>(tot, lig, T);
    ex *= o;
    if constexpr (2 * D < G) tot *= o;
    excl_levels<G, 2 * D>(ex, tot, lig, T);
  }
}
template <int G>
__device__ __forceinline__ float grp_excl(float v, int lig, int T) {
  float ex = 1.f, tot = v;
  excl_levels<G>(ex, tot, lig, T);
  return ex;
}

template <int G, int D = 1>
__device__ __forceinline__ void excl_levels_c(cf& ex, cf& tot, int lig, int T) {
  if constexpr (D < G) {
    const cf o{grp_xchg<D>(tot.r, lig, T), grp_xchg<D>(tot.i, lig, T)};
    ex = cmul(ex, o);
    if constexpr (2 * D < G) tot = cmul(tot, o);
    excl_levels_c<G, 2 * D>(ex, tot, lig, T);
  }
}
template <int G>
__device__ __forceinline__ cf grp_excl_c(cf v, int lig, int T) {
  cf ex{1.f, 0.f}, tot = v;
  excl_levels_c<G>(ex, tot, lig, T);
  return ex;
}

// ------------------------------------------------------ one constraint, one restart
// Literal i of the pair's constraint is handled by group lane i / J, slot i % J.

// What a lane needs from memory for its pair: the literal codes of its J
// slots (-1 past the constraint's end or past the segment), the class and the
// weight.  Fetching is split from computing so that the next pair's loads are
// in flight while the current pair is evaluated.
template <int J>
struct Fetched {
  int code[J];
  int cls;
  float w;
};

template <int J, int KMAX>
__device__ __forceinline__ void fetch_pair(const ProblemDev& P, const Segment& S, int c_local, int lig,
                                           Fetched<J>& f) {
  // A lane past the segment fetches its last pair (valid memory, no branch); the
  // caller skips evaluating it.
  const int cl = min(c_local, S.c_count - 1);
  // Buffer loads: the slot's column offset is wave-uniform (scalar soffset) and
  // the lane's offset is one 32-bit register shared by every slot.
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(P.litT + S.lit_base), (short)0, KMAX * S.c_count * 4, 0x00020000);
  const unsigned voff = ((unsigned)(lig * J) * (unsigned)S.c_count + (unsigned)cl) * 4u;
#pragma unroll
  for (int j = 0; j < J; ++j) f.code[j] = __builtin_amdgcn_raw_buffer_load_b32(rs, voff, j * S.c_count * 4, 0);
  const int c = S.c_begin + cl;
  f.cls = S.cls_fixed >= 0 ? S.cls_fixed : P.c_cls[c];
  f.w = P.unit_weights ? 1.f : P.c_w[c];
}

// Literal decode: LDS element of (variable, restart t) and the sign bit, which
// is XORed onto x (y = s x) and onto the gradient term (dF/dx = s dF/dy).
// Byte offset of (variable, restart t) in an array of 4-byte elements laid out
// [variable][T]: shifting by log2 T + 2 >= 2 drops the sign bit.  The gradient
// array uses the same offset scaled by its element size.
__device__ __forceinline__ unsigned lit_off(int code, int logT, int t) {
  return ((unsigned)code << (logT + 2)) | ((unsigned)t << 2);
}
// x is the first array of the kernels' dynamic LDS, which starts at LDS
// address 0 (the kernels hold no static LDS; the host checks this), so the
// byte offset is the address itself: no base add per literal.
__device__ __forceinline__ float x_at(const float*, unsigned off) {
  return *reinterpret_cast<const __attribute__((address_space(3))) float*>((size_t)off);
}
template <class AT>
__device__ __forceinline__ AT* g_at(AT* gs, unsigned off) {
  return reinterpret_cast<AT*>(reinterpret_cast<char*>(gs) + off * (unsigned)(sizeof(AT) / 4));
}

// Where a pair's per-literal gradient terms go: the tile's fixed-point LDS
// accumulator (GradSink), or a per-lane sum of squares (SquareSink, for the
// per-constraint gradient statistics).
// Terms of pad slots (code of a pad row, variable >= n) go to the pad row's
// accumulator, which is never read; the statistics sink skips them.
template <class AT>
struct GradSink {
  AT* gs;
  __device__ __forceinline__ void add(unsigned off, float v, int) { FixedAcc<AT>::add(g_at(gs, off), v); }
};
struct SquareSink {
  float acc;
  int n;
  __device__ __forceinline__ void add(unsigned, float v, int code) {
    acc = ((code & 0x7fffffff) < n) ? fmaf(v, v, acc) : acc;
  }
};
__device__ __forceinline__ unsigned lit_sign(int code) { return (unsigned)code & 0x80000000u; }
__device__ __forceinline__ float flip(float v, unsigned sb) { return __uint_as_float(__float_as_uint(v) ^ sb); }

// Product kinds: FE - c0 = c1 prod (a + b y) [+ c2 prod (1 - y)/2];
// dFE/dy_i = c1 b prod_{j != i} (a + b y_j) [- c2/2 prod_{j != i} (1 - y_j)/2].
struct ProdParams {
  float a, b, c1, c2;
};

__device__ __forceinline__ ProdParams prod_params(kptr<ClassRec> classes, int cls) {
  return {classes[cls].a, classes[cls].b, classes[cls].c1, classes[cls].c2};
}

// The same with the fixed-point scales folded in once per class: f = c fsc for
// the objective, s1 = c1 b gsc and s2 = -c2/2 gsc for the gradient.  The scales
// are powers of two, so every product equals the one formed by scaling last.
struct ProdConsts {
  float a, b, f1, f2, s1, s2;
};

__device__ __forceinline__ ProdConsts prod_consts(kptr<ClassRec> classes, int cls, float gsc, float fsc) {
  const float a = classes[cls].a, b = classes[cls].b, c1 = classes[cls].c1, c2 = classes[cls].c2;
  return {a, b, c1 * fsc, c2 * fsc, c1 * b * gsc, -0.5f * c2 * gsc};
}

// Slots past a constraint's end code a pad row whose factor is exactly 1 (the
// sign is chosen by the planner), except the second node of PROD2, which a
// select sets to 1: every slot is read and processed without a branch.
template <int NN, int KMAX, int G, class SK>
__device__ __forceinline__ void prod_pair(const Fetched<KMAX / G>& fp, int lig, int t, int logT, int n,
                                          const float* xs, SK& sink, float& fchunk, float gsc, float fsc,
                                          const ProdParams& pp) {
  constexpr int J = KMAX / G;
  constexpr bool kExact = KMAX <= 8;  // buckets up to 8 hold a single length
  const int T = 1 << logT;
  const float a1 = pp.a, b1 = pp.b, c1 = pp.c1, c2 = pp.c2;

  unsigned el[J];
  float f1[J], f2[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int code = fp.code[j];
    el[j] = lit_off(code, logT, t);
    const float y = flip(x_at(xs, el[j]), lit_sign(code));
    f1[j] = fmaf(b1, y, a1);
    f2[j] = 1.f;
    if constexpr (NN == 2) f2[j] = (kExact || (code & 0x7fffffff) < n) ? fmaf(-0.5f, y, 0.5f) : 1.f;
  }
  float pre1[J], pre2[J];
  float run1 = 1.f, run2 = 1.f;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    pre1[j] = run1;
    run1 *= f1[j];
    if constexpr (NN == 2) {
      pre2[j] = run2;
      run2 *= f2[j];
    }
  }
  // the other lanes' products
  const float ex1 = grp_excl<G>(run1, lig, T);
  float ex2 = 1.f;
  if constexpr (NN == 2) ex2 = grp_excl<G>(run2, lig, T);
  if (lig == 0) {
    float fe = c1 * (run1 * ex1);
    if constexpr (NN == 2) fe = fmaf(c2, run2 * ex2, fe);
    fchunk = fmaf(fp.w * fsc, fe, fchunk);
  }
  // the suffix products start at the gradient scales, so each literal's term
  // is one product: prefix_j * (scale * suffix_j)
  float suf1 = c1 * b1 * (fp.w * gsc) * ex1;
  float suf2 = -0.5f * c2 * (fp.w * gsc) * ex2;
#pragma unroll
  for (int j = J - 1; j >= 0; --j) {
    float g = pre1[j] * suf1;
    suf1 *= f1[j];
    if constexpr (NN == 2) {
      g = fmaf(pre2[j], suf2, g);
      suf2 *= f2[j];
    }
    sink.add(el[j], flip(g, lit_sign(fp.code[j])), fp.code[j]);
  }
}

// Generic kind: FE - chat_0 = sum_{m=1}^{M} Re(2 chat_m Q_m) [+ chat_{K/2} prod y];
// dFE/dy_i = sum_m Re(2 chat_m beta_m prod_{j != i}(alpha_m + beta_m y_j)) [+ chat_{K/2} prod_{j != i} y_j].
// cls is the pair's class; when the caller passes a wave-uniform value the class
// record and the node table are read with scalar loads.
template <int KMAX, int G, class SK>
__device__ __forceinline__ void dft_pair(const ProblemDev& P, int m_max, int cls, const Fetched<KMAX / G>& fp,
                                         int lig, int t, int logT, const float* xs, SK& sink, float& fchunk,
                                         float gsc, float fsc) {
  constexpr int J = KMAX / G;
  constexpr bool kExact = KMAX <= 8;  // buckets up to 8 hold a single length
  const int T = 1 << logT;
  kptr<ClassRec> classes = kconst(P.classes);
  const int nyquist = classes[cls].nyquist;
  const float cn = classes[cls].c1;
  const int node_off = classes[cls].node_off;
  const int nn = classes[cls].n_nodes;

  unsigned el[J];
  float y[J], g[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int code = fp.code[j];
    el[j] = lit_off(code, logT, t);  // pad slots read y = 1: factor alpha + beta = 1 exactly
    y[j] = flip(x_at(xs, el[j]), lit_sign(code));
    g[j] = 0.f;
  }
  float fe = 0.f;
  if (nyquist) {  // real node omega^(K/2) = -1: factor y, padded slots hold y = 1
    float pre[J];
    float run = 1.f;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      pre[j] = run;
      run *= y[j];
    }
    const float ex = grp_excl<G>(run, lig, T);
    fe = cn * (run * ex);
    const float sc = cn * ex;
    float suf = 1.f;
#pragma unroll
    for (int j = J - 1; j >= 0; --j) {
      g[j] = sc * pre[j] * suf;
      suf *= y[j];
    }
  }
  kptr<NodeRec> nd = kconst(P.nodes) + node_off;
  for (int mm = 0; mm < m_max; ++mm) {
    if (mm < nn) {
      const NodeRec N{nd[mm].ar, nd[mm].ai, nd[mm].br, nd[mm].bi, nd[mm].wr, nd[mm].wi, nd[mm].gr, nd[mm].gi};
      cf pre[J];
      cf run{1.f, 0.f};
#pragma unroll
      for (int j = 0; j < J; ++j) {
        pre[j] = run;
        const cf f{fmaf(N.br, y[j], N.ar), fmaf(N.bi, y[j], N.ai)};
        run = cmul(run, f);
      }
      const cf ex = grp_excl_c<G>(run, lig, T);  // the other lanes' node products
      const cf tot = cmul(run, ex);
      fe = fmaf(N.wr, tot.r, fmaf(-N.wi, tot.i, fe));
      // The gradient of literal j is Re(gw * prefix_j * suffix_j), gw the node's
      // gradient weight: carrying S_j = gw * (other lanes) * (lane suffix)_j down
      // the literals leaves one real part of a product per literal.
      cf S = cmul(cf{N.gr, N.gi}, ex);
#pragma unroll
      for (int j = J - 1; j >= 0; --j) {
        g[j] = fmaf(pre[j].r, S.r, fmaf(-pre[j].i, S.i, g[j]));  // Re(pre_j * S_j)
        const cf f{fmaf(N.br, y[j], N.ar), fmaf(N.bi, y[j], N.ai)};
        S = cmul(S, f);
      }
    }
  }
  if (lig == 0) fchunk = fmaf(fp.w * fsc, fe, fchunk);
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const float gv = (fp.w * gsc) * g[j];
    sink.add(el[j], flip(gv, lit_sign(fp.code[j])), fp.code[j]);
  }
}

// Waves claim chunks of a segment's constraints from an LDS counter (one chunk
// = the constraints one wave covers: 64 / (G T)), so heavy and light items
// spread over the waves as they finish; segments are ordered heaviest first.
// PMF kind (k <= 8, one lane per pair).  With pi_i = 1/2 - h y_i the
// probability that literal i adds to the count C, the truncated distribution
// q_c = Pr[C = c], c < 4, follows q <- q (1 - pi_i) + shift(q) pi_i; the value
// is sum_c d_c q_c.  Reverse mode: with lambda = d after the last literal,
// dFE/dpi_i = sum_c pre_i[c] (lambda_{c+1} - lambda_c) (lambda_4 = 0) where pre_i
// is q before literal i, then lambda_c <- lambda_c + pi_i (lambda_{c+1} - lambda_c).
// Every update is a convex combination, so no cancellation arises.
// W: counts kept, the widest window of the segment (coefficients past a class's
// own window are zero, so a wider W changes no value).
template <int KMAX, int W, class SK>
__device__ __forceinline__ void pmf_pair(const ProblemDev& P, int cls, const Fetched<KMAX>& fp, int t, int logT,
                                         const float* xs, SK& sink, float& fchunk, float gsc, float fsc) {
  constexpr int J = KMAX;  // buckets up to 8 hold a single length
  static_assert(W >= 1 && W <= kPmfWindow, "window");
  kptr<ClassRec> classes = kconst(P.classes);
  kptr<NodeRec> nd = kconst(P.nodes) + classes[cls].node_off;
  const float dall[kPmfWindow] = {nd[0].ar, nd[0].ai, nd[0].br, nd[0].bi};
  float d[W];
#pragma unroll
  for (int c = 0; c < W; ++c) d[c] = dall[c];
  const float h = nd[0].wr;

  unsigned el[J];
  float pi[J], pre[J][W];
  float q[W];
  q[0] = 1.f;
#pragma unroll
  for (int c = 1; c < W; ++c) q[c] = 0.f;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    el[j] = lit_off(fp.code[j], logT, t);
    const float y = flip(x_at(xs, el[j]), lit_sign(fp.code[j]));
    pi[j] = fmaf(-h, y, 0.5f);
#pragma unroll
    for (int c = 0; c < W; ++c) pre[j][c] = q[c];
#pragma unroll
    for (int c = W - 1; c >= 1; --c) q[c] = fmaf(pi[j], q[c - 1] - q[c], q[c]);
    q[0] = fmaf(-pi[j], q[0], q[0]);
  }
  float fe = 0.f;
#pragma unroll
  for (int c = 0; c < W; ++c) fe = fmaf(d[c], q[c], fe);
  fchunk = fmaf(fp.w * fsc, fe, fchunk);
  // dFE/dy_i = -h dFE/dpi_i
  const float coef = -h * (fp.w * gsc);
  float* lam = d;
#pragma unroll
  for (int j = J - 1; j >= 0; --j) {
    float diff[W], gp = 0.f;
#pragma unroll
    for (int c = 0; c < W; ++c) {
      diff[c] = (c + 1 < W ? lam[c + 1] : 0.f) - lam[c];
      gp = fmaf(pre[j][c], diff[c], gp);
    }
#pragma unroll
    for (int c = 0; c < W; ++c) lam[c] = fmaf(pi[j], diff[c], lam[c]);
    sink.add(el[j], flip(coef * gp, lit_sign(fp.code[j])), fp.code[j]);
  }
}

// Lane exchange inside a pair's lane group: the value of the lane at xor
// distance dist.  Distances 1 and 2 are DPP quad permutations (one VALU move,
// no LDS traffic); longer ones are wave shuffles.
template <int N>
__device__ __forceinline__ void xor_exchange(const float (&src)[N], float (&dst)[N], int dist) {
  if (dist == 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) dst[i] = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(src[i]), 0xB1, 0xf, 0xf, true));
  } else if (dist == 2) {
#pragma unroll
    for (int i = 0; i < N; ++i) dst[i] = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(src[i]), 0x4E, 0xf, 0xf, true));
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) dst[i] = __shfl_xor(src[i], dist);
  }
}

// Truncated count recursion over N literals with event probabilities pi:
// q(c) = Pr[count = c] for c < M, and pre[j] = q before literal j (counts
// 0..j; entries past j are zero and not kept).
template <int N, int M>
__device__ __forceinline__ void count_forward(const float* pi, float (&pre)[N][M], float (&q)[M]) {
  q[0] = 1.f;
#pragma unroll
  for (int c = 1; c < M; ++c) q[c] = 0.f;
#pragma unroll
  for (int j = 0; j < N; ++j) {
#pragma unroll
    for (int c = 0; c < M; ++c)
      if (c <= j) pre[j][c] = q[c];
#pragma unroll
    for (int c = M - 1; c >= 1; --c)
      if (c <= j + 1) q[c] = fmaf(pi[j], q[c - 1] - q[c], q[c]);
    q[0] = fmaf(-pi[j], q[0], q[0]);
  }
}

// Reverse mode of count_forward for an objective sum_c q(c) lam(c) (lam past
// M - 1 is zero): gp[j] = d objective / d pi_j.  lam is consumed.
template <int N, int M>
__device__ __forceinline__ void count_adjoint(const float* pi, const float (&pre)[N][M], float (&lam)[M],
                                              float* gp) {
#pragma unroll
  for (int j = N - 1; j >= 0; --j) {
    float g = 0.f;
#pragma unroll
    for (int c = 0; c < M; ++c) {
      if (c <= j) {
        const float diff = (c + 1 < M ? lam[c + 1] : 0.f) - lam[c];
        g = fmaf(pre[j][c], diff, g);
        lam[c] = fmaf(pi[j], diff, lam[c]);
      }
    }
    gp[j] = g;
  }
}

// PMF kind for constraints of 9 to 32 literals whose spectrum is constant past
// a window of at most KMAX/2 counts at one end (thresholds near the middle such
// as at-least-ceil(k/2), exactly-one, at-most-one, exactly-kappa near an end).
// The pair's G lanes hold J literals each, in two halves of J/2.  Each half
// runs the truncated count recursion of the PMF kind, giving its count
// distribution qa, qb; the lane's own count has q = qa * qb (convolution).  The
// count over the other lanes of the group has the distribution E, the
// truncated convolution of their q (G = 2: the partner's q; G = 4: the
// partner's q convolved with the other pair's convolved total), obtained by
// lane exchanges.  With D(c) = sum_b d_{c+b} E(b) (d zero past the window),
// FE = c0 + sum_c q(c) D(c) in every lane of the group; as a function of half
// a's distribution, FE = c0 + sum_a qa(a) DA(a) with DA(a) = sum_b qb(b) D(a+b),
// so each literal's gradient is the adjoint of its half's recursion started
// from DA (or DB).  Every step adds products of probabilities: no
// cancellation, and about (J + W) operations per literal against about 14 per
// node and literal (k/2 nodes) on the DFT path.
// Class data (node table entries read as floats): d_0..d_31 (zero past the
// window), h at 32, and at 33 a flag for threshold windows (d constant on the
// window [0, w), w the class's window).
template <int KMAX, int G, class SK>
__device__ __forceinline__ void pmfg_pair(const ProblemDev& P, int cls, const Fetched<KMAX / G>& fp, int lig, int t,
                                          int logT, const float* xs, SK& sink, float& fchunk, float gsc, float fsc) {
  constexpr int J = KMAX / G;
  constexpr int H = J / 2;                    // literals per half
  constexpr int MH = H + 1;                   // counts of a half (never truncated: H + 1 <= W)
  constexpr int W = KMAX / 2;                 // widest window of the bucket
  constexpr int WL = J + 1 < W ? J + 1 : W;   // counts of one lane kept
  static_assert(G == 2 || G == 4, "lane groups of 2 or 4 (8: pmfg8_pair)");
  static_assert(J % 2 == 0 && MH <= W, "halves");
  const int T = 1 << logT;
  kptr<ClassRec> classes = kconst(P.classes);
  kptr<float> dt = reinterpret_cast<kptr<float>>(kconst(P.nodes) + classes[cls].node_off);
  float d[W];
#pragma unroll
  for (int c = 0; c < W; ++c) d[c] = dt[c];
  const float h = dt[32];

  float pi[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int code = fp.code[j];  // a pad slot reads y = 2h: pi = 0, it adds nothing to the count
    pi[j] = fmaf(-h, flip(x_at(xs, lit_off(code, logT, t)), lit_sign(code)), 0.5f);
  }
  float prea[H][MH], preb[H][MH], qa[MH], qb[MH];
  count_forward<H, MH>(pi, prea, qa);
  count_forward<H, MH>(pi + H, preb, qb);
  float q[WL];
#pragma unroll
  for (int c = 0; c < WL; ++c) {
    float acc = 0.f;
#pragma unroll
    for (int a = 0; a < MH; ++a)
      if (c - a >= 0 && c - a < MH) acc = fmaf(qa[a], qb[c - a], acc);
    q[c] = acc;
  }

  // D(c) = sum_b d_{c+b} E(b)
  float D[WL];
  if constexpr (G == 2) {
    float e[WL];
    xor_exchange(q, e, T);
#pragma unroll
    for (int c = 0; c < WL; ++c) {
      float acc = 0.f;
#pragma unroll
      for (int b = 0; b < WL; ++b)
        if (c + b < W) acc = fmaf(d[c + b], e[b], acc);
      D[c] = acc;
    }
  } else {
    float x1[WL];
    xor_exchange(q, x1, T);  // partner in the same half of the group
    float y2[W];             // that half's total count, truncated
#pragma unroll
    for (int c = 0; c < W; ++c) {
      float acc = 0.f;
#pragma unroll
      for (int a = 0; a < WL; ++a)
        if (c - a >= 0 && c - a < WL) acc = fmaf(q[a], x1[c - a], acc);
      y2[c] = acc;
    }
    float z[W];
    xor_exchange(y2, z, 2 * T);  // the other half's total
    // dz(j) = sum_b d_{j+b} z(b); D(c) = sum_a x1(a) dz(c + a)
    float dz[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
      float acc = 0.f;
#pragma unroll
      for (int b = 0; b < W; ++b)
        if (j + b < W) acc = fmaf(d[j + b], z[b], acc);
      dz[j] = acc;
    }
#pragma unroll
    for (int c = 0; c < WL; ++c) {
      float acc = 0.f;
#pragma unroll
      for (int a = 0; a < WL; ++a)
        if (c + a < W) acc = fmaf(x1[a], dz[c + a], acc);
      D[c] = acc;
    }
  }
  // per half: DA(a) = sum_b qb(b) D(a+b), DB(b) = sum_a qa(a) D(a+b)
  float DA[MH], DB[MH];
#pragma unroll
  for (int a = 0; a < MH; ++a) {
    float sa = 0.f, sb = 0.f;
#pragma unroll
    for (int b = 0; b < MH; ++b)
      if (a + b < WL) {
        sa = fmaf(qb[b], D[a + b], sa);
        sb = fmaf(qa[b], D[a + b], sb);
      }
    DA[a] = sa;
    DB[a] = sb;
  }
  float fe = 0.f;
#pragma unroll
  for (int a = 0; a < MH; ++a) fe = fmaf(qa[a], DA[a], fe);
  if (lig == 0) fchunk = fmaf(fp.w * fsc, fe, fchunk);

  // dFE/dy_j = -h dFE/dpi_j
  float gp[J];
  count_adjoint<H, MH>(pi, prea, DA, gp);
  count_adjoint<H, MH>(pi + H, preb, DB, gp + H);
  const float coef = -h * (fp.w * gsc);
#pragma unroll
  for (int j = J - 1; j >= 0; --j)
    sink.add(lit_off(fp.code[j], logT, t), flip(coef * gp[j], lit_sign(fp.code[j])), fp.code[j]);
}

// Count distribution of N literals (probabilities pi), truncated to M counts,
// without keeping the intermediate distributions.
template <int N, int M>
__device__ __forceinline__ void count_only(const float* pi, float (&q)[M]) {
  q[0] = 1.f;
#pragma unroll
  for (int c = 1; c < M; ++c) q[c] = 0.f;
#pragma unroll
  for (int j = 0; j < N; ++j) {
#pragma unroll
    for (int c = M - 1; c >= 1; --c)
      if (c <= j + 1) q[c] = fmaf(pi[j], q[c - 1] - q[c], q[c]);
    q[0] = fmaf(-pi[j], q[0], q[0]);
  }
}

// Truncated convolution r = (u * v) restricted to counts < NR.
template <int NU, int NV, int NR>
__device__ __forceinline__ void conv_trunc(const float (&u)[NU], const float (&v)[NV], float (&r)[NR]) {
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    float acc = 0.f;
#pragma unroll
    for (int a = 0; a < NU; ++a)
      if (c - a >= 0 && c - a < NV) acc = fmaf(u[a], v[c - a], acc);
    r[c] = acc;
  }
}

// The lane at xor distance 4 T in the lane's group of eight.  With T = 1 the
// group is an 8-lane half-row: the lower quad reads 4 lanes up, the upper quad 4
// lanes down (two DPP row shifts and a select); otherwise a wave shuffle.  The
// partner is the same lane either way, so results do not depend on T (the four
// lanes of a quad hold totals summed in different orders, which may differ in
// the last bit).
template <int N>
__device__ __forceinline__ void other_quad(const float (&src)[N], float (&dst)[N], int T, int lig) {
  if (T == 1) {
    const bool upper = (lig & 4) != 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const float up = row_shl<4>(src[i]), dn = row_shr<4>(src[i]);
      dst[i] = upper ? dn : up;
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) dst[i] = __shfl_xor(src[i], 4 * T);
  }
}

// PMF kind for 33 to 48 literals (lane groups of G = 8, J = KMAX/8 literals per
// lane, window up to W = KMAX/2 counts): as pmfg_pair with one more level of the
// butterfly, the other quad's total z4.  E = x1 * z2 * z4 is not formed; with
// R4(j) = sum_b d_{j+b} z4(b) and R2(j) = sum_a z2(a) R4(j+a),
// D(c) = sum_a x1(a) R2(c+a).  For a threshold window (d = d_0 on [0, w)),
// R4(j) = d_0 S(w - j), S(m) the sum of z4 below m, read at the wave-uniform
// offset W - w by a barrel shift of uniform branches instead of the W^2/2
// products of the general correlation.  To stay within the register budget the
// lane's local distributions are computed twice: once without their
// intermediate distributions for the butterfly, then with them for the adjoint.
template <int KMAX, class SK>
__device__ __forceinline__ void pmfg8_pair(const ProblemDev& P, int cls, const Fetched<KMAX / 8>& fp, int lig,
                                           int t, int logT, const float* xs, SK& sink, float& fchunk, float gsc,
                                           float fsc) {
  constexpr int J = KMAX / 8;
  constexpr int H = J / 2;
  constexpr int MH = H + 1;
  constexpr int W = KMAX / 2;
  constexpr int WL = J + 1;            // counts of one lane (J + 1 <= W)
  constexpr int W2 = 2 * WL - 1;       // counts of a pair (2 J + 1 <= W)
  static_assert(J % 2 == 0 && W2 <= W, "shape");
  const int T = 1 << logT;
  kptr<ClassRec> classes = kconst(P.classes);
  kptr<float> dt = reinterpret_cast<kptr<float>>(kconst(P.nodes) + classes[cls].node_off);
  const int w = classes[cls].nyquist;
  const float h = dt[32];
  const bool thr = dt[33] != 0.f;

  float pi[J];
#pragma unroll
  for (int j = 0; j < J; ++j)
    pi[j] = fmaf(-h, flip(x_at(xs, lit_off(fp.code[j], logT, t)), lit_sign(fp.code[j])), 0.5f);

  // butterfly over the group: D(c) for the lane's local count c < WL
  float D[WL];
  {
    float x1[WL];
    {
      float qa[MH], qb[MH], q[WL];
      count_only<H, MH>(pi, qa);
      count_only<H, MH>(pi + H, qb);
      conv_trunc(qa, qb, q);
      xor_exchange(q, x1, T);
      float y2[W2];
      conv_trunc(q, x1, y2);
      float z2[W2];
      xor_exchange(y2, z2, 2 * T);
      float R4[W];
      {
        float y4[W];
        conv_trunc(y2, z2, y4);
        float z4[W];
        other_quad(y4, z4, T, lig);
        if (thr) {
          // A(i) = sum_{b < W - i} z4(b), then shifted left by W - w: A(j) -> S(w - j)
          float A[W];
          float run = 0.f;
#pragma unroll
          for (int i = W - 1; i >= 0; --i) {
            run += z4[W - 1 - i];
            A[i] = run;
          }
          const int sft = W - w;  // wave-uniform, 0 <= sft < W
#pragma unroll
          for (int k = 1; k < W; k <<= 1) {
            if (sft & k) {
#pragma unroll
              for (int i = 0; i < W; ++i) A[i] = i + k < W ? A[i + k] : 0.f;
            }
          }
          const float d0 = dt[0];
#pragma unroll
          for (int j = 0; j < W; ++j) R4[j] = d0 * A[j];
        } else {
#pragma unroll
          for (int j = 0; j < W; ++j) {
            float acc = 0.f;
#pragma unroll
            for (int b = 0; b < W; ++b)
              if (j + b < W) acc = fmaf(dt[j + b], z4[b], acc);
            R4[j] = acc;
          }
        }
      }
      float R2[W2];
#pragma unroll
      for (int j = 0; j < W2; ++j) {
        float acc = 0.f;
#pragma unroll
        for (int a = 0; a < W2; ++a)
          if (j + a < W) acc = fmaf(z2[a], R4[j + a], acc);
        R2[j] = acc;
      }
#pragma unroll
      for (int c = 0; c < WL; ++c) {
        float acc = 0.f;
#pragma unroll
        for (int a = 0; a < WL; ++a) acc = fmaf(x1[a], R2[c + a], acc);
        D[c] = acc;
      }
    }
  }

  // the lane's halves again, with their intermediate distributions
  float prea[H][MH], preb[H][MH], qa[MH], qb[MH];
  count_forward<H, MH>(pi, prea, qa);
  count_forward<H, MH>(pi + H, preb, qb);
  float DA[MH], DB[MH];
#pragma unroll
  for (int a = 0; a < MH; ++a) {
    float sa = 0.f, sb = 0.f;
#pragma unroll
    for (int b = 0; b < MH; ++b) {
      sa = fmaf(qb[b], D[a + b], sa);
      sb = fmaf(qa[b], D[a + b], sb);
    }
    DA[a] = sa;
    DB[a] = sb;
  }
  float fe = 0.f;
#pragma unroll
  for (int a = 0; a < MH; ++a) fe = fmaf(qa[a], DA[a], fe);
  if (lig == 0) fchunk = fmaf(fp.w * fsc, fe, fchunk);
  float gp[J];
  count_adjoint<H, MH>(pi, prea, DA, gp);
  count_adjoint<H, MH>(pi + H, preb, DB, gp + H);
  const float coef = -h * (fp.w * gsc);
#pragma unroll
  for (int j = J - 1; j >= 0; --j)
    sink.add(lit_off(fp.code[j], logT, t), flip(coef * gp[j], lit_sign(fp.code[j])), fp.code[j]);
}

// Per-lane objective partial sums (exact integers): `own` for restart
// lane mod T; `even` and `odd` for restarts 2 t2 and 2 t2 + 1 of the paths that
// give a lane two adjacent restarts (t2 = lane mod T/2).
struct ObjAcc {
  long long own, even, odd;
};

// Two restarts per lane (short product constraints, tiles of T >= 2): the
// codes, the address decode, the claim and the loop control are shared by two
// literal-evaluations; x of both restarts arrives in one 8-byte LDS read and the
// second gradient term goes to the next LDS word.
template <int NN, int KMAX, bool UW, class AT>
__device__ __forceinline__ void prod_pair_r2(const Fetched<KMAX>& fp, int t2, int logT, const float* xs, AT* gs,
                                             float& fca, float& fcb, const ProdConsts& pc) {
  constexpr int J = KMAX;  // one lane per pair, every slot filled (buckets up to 8 hold one length)
  const float a1 = pc.a, b1 = pc.b;
  unsigned el[J];
  float fa1[J], fb1[J], fa2[J], fb2[J];
  // the literal's sign goes onto the node coefficient once for both restarts:
  // b (s x) = (s b) x exactly (and below onto each gradient term)
#pragma unroll
  for (int j = 0; j < J; ++j) {
    el[j] = lit_off(fp.code[j], logT, 2 * t2);
    const float2 xv = *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(xs) + el[j]);
    const unsigned sb = lit_sign(fp.code[j]);
    const float bj = flip(b1, sb);
    fa1[j] = fmaf(bj, xv.x, a1);
    fb1[j] = fmaf(bj, xv.y, a1);
    if constexpr (NN == 2) {
      const float hj = flip(-0.5f, sb);
      fa2[j] = fmaf(hj, xv.x, 0.5f);
      fb2[j] = fmaf(hj, xv.y, 0.5f);
    }
  }
  float pa1[J], pb1[J], pa2[J], pb2[J];
  float ra1 = 1.f, rb1 = 1.f, ra2 = 1.f, rb2 = 1.f;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    pa1[j] = ra1;
    pb1[j] = rb1;
    ra1 *= fa1[j];
    rb1 *= fb1[j];
    if constexpr (NN == 2) {
      pa2[j] = ra2;
      pb2[j] = rb2;
      ra2 *= fa2[j];
      rb2 *= fb2[j];
    }
  }
  // objective w (c1 P1 [+ c2 P2]) fsc; unit weights: one FMA per restart and node
  float s1 = pc.s1, s2 = pc.s2;
  if constexpr (UW) {
    if constexpr (NN == 2) {
      fca = fmaf(pc.f2, ra2, fca);
      fcb = fmaf(pc.f2, rb2, fcb);
    }
    fca = fmaf(pc.f1, ra1, fca);
    fcb = fmaf(pc.f1, rb1, fcb);
  } else {
    float fea = pc.f1 * ra1, feb = pc.f1 * rb1;
    if constexpr (NN == 2) {
      fea = fmaf(pc.f2, ra2, fea);
      feb = fmaf(pc.f2, rb2, feb);
    }
    fca = fmaf(fp.w, fea, fca);
    fcb = fmaf(fp.w, feb, fcb);
    s1 *= fp.w;
    s2 *= fp.w;
  }
  // the suffix products start at the gradient scales (one product per term)
  float sa1 = s1, sb1 = s1, sa2 = s2, sb2 = s2;
#pragma unroll
  for (int j = J - 1; j >= 0; --j) {
    const unsigned sg = lit_sign(fp.code[j]);  // dF/dx = s dF/dy
    float ga = pa1[j] * sa1, gb = pb1[j] * sb1;
    sa1 *= fa1[j];
    sb1 *= fb1[j];
    if constexpr (NN == 2) {
      ga = fmaf(pa2[j], sa2, ga);
      gb = fmaf(pb2[j], sb2, gb);
      sa2 *= fa2[j];
      sb2 *= fb2[j];
    }
    AT* gp = g_at(gs, el[j]);
    FixedAcc<AT>::add(gp, flip(ga, sg));
    FixedAcc<AT>::add(gp + 1, flip(gb, sg));
  }
}

// Pairs each lane takes per claim: short product constraints are cheap, so a
// lane takes several of them per claim, which amortises the claim, the fetch
// addressing and the loop control over more literals.
// Kernels built for long constraints (MAXB above the 8-literal bucket) keep one
// pair per lane: their register budget goes to the long groups.
template <int KIND, int J, int MAXB>
constexpr int pairs_per_lane() {
  return (KIND == KIND_DFT || KIND == KIND_PMF || MAXB > kMaxbShort) ? 1 : (J <= 4 ? 4 : (J <= 8 ? 2 : 1));
}

template <int J, int U>
struct FetchedU {
  Fetched<J> p[U];
};

// The two-restarts-per-lane variant of run_segment for short product kinds.
template <int KIND, int KMAX, bool UW, class AT>
__device__ __forceinline__ void run_segment_r2(const ProblemDev& P, const Segment& S, const float* xs, AT* gs,
                                               ObjAcc& facc, float gsc, float fsc, int tid, int logT, int* ctr) {
  constexpr int J = KMAX;
  constexpr int U = J <= 4 ? 2 : 1;
  asm volatile("" : "+v"(tid));
  const int lane = tid & (kWave - 1);
  const int t2 = lane & ((1 << (logT - 1)) - 1);
  const int sub = lane >> (logT - 1);
  const int per_wave = kWave >> (logT - 1);
  kptr<ClassRec> classes = kconst(P.classes);
  const bool uni = S.cls_fixed >= 0;
  ProdConsts pc_uni{};
  if (uni) pc_uni = prod_consts(classes, S.cls_fixed, gsc, fsc);
  auto claim = [&]() {
    int b = 0;
    if (lane == 0) b = atomicAdd(ctr, U * per_wave);
    return __builtin_amdgcn_readfirstlane(b);
  };
  auto fetch = [&](int b, FetchedU<J, U>& f) {
#pragma unroll
    for (int u = 0; u < U; ++u) fetch_pair<J, KMAX>(P, S, b + u * per_wave + sub, 0, f.p[u]);
  };
  int base = claim();
  FetchedU<J, U> cur;
  fetch(base, cur);
  while (base < S.c_count) {
    const int nbase = claim();
    FetchedU<J, U> nxt;
    fetch(nbase, nxt);
    float fca = 0.f, fcb = 0.f;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b_u = base + u * per_wave;
      if (u > 0 && b_u >= S.c_count) break;
      const Fetched<J>& fp = cur.p[u];
      const bool valid = b_u + sub < S.c_count;
      const int c0 = __builtin_amdgcn_readfirstlane(fp.cls);
      const bool chunk_uni = uni || !__any(valid && fp.cls != c0);
      if (valid) {
        const ProdConsts pc = uni ? pc_uni : prod_consts(classes, chunk_uni ? c0 : fp.cls, gsc, fsc);
        prod_pair_r2<KIND == KIND_PROD2 ? 2 : 1, KMAX, UW>(fp, t2, logT, xs, gs, fca, fcb, pc);
      }
    }
    facc.even += fixed_term(fca);
    facc.odd += fixed_term(fcb);
    cur = nxt;
    base = nbase;
  }
}

// Per-constraint gradient statistics (statistics kernel only): 64-bit
// fixed-point sums at scale 2^s of sum_i (dFE_c/dy_i)^2, planned order.
struct StatsOut {
  unsigned long long* acc;
  float scale;
};

template <int KIND, int KMAX, int MAXB, class AT, bool ST = false>
__device__ __forceinline__ void run_segment(const ProblemDev& P, const Segment& S, const float* xs, AT* gs,
                                            ObjAcc& facc, float gsc, float fsc, int tid, int logT, int* ctr,
                                            StatsOut so = {}) {
  if constexpr (!ST && (KIND == KIND_PROD1 || KIND == KIND_PROD2) && MAXB <= kMaxbShort && KMAX <= 8) {
    if (logT >= 1) {
      // unit weights (a problem-wide flag): no weight fetch or multiply
      if (P.unit_weights)
        run_segment_r2<KIND, KMAX, true>(P, S, xs, gs, facc, gsc, fsc, tid, logT, ctr);
      else
        run_segment_r2<KIND, KMAX, false>(P, S, xs, gs, facc, gsc, fsc, tid, logT, ctr);
      return;
    }
  }
  constexpr int G = group_size(KIND, KMAX);
  constexpr int LG = Log2<G>::v;
  constexpr int J = KMAX / G;
  constexpr int U = pairs_per_lane<KIND, J, MAXB>();
  // keep the lane-index arithmetic inside the segment: hoisting it out of the
  // step loop for every instantiation at once exhausts the register budget
  asm volatile("" : "+v"(tid));
  const int lane = tid & (kWave - 1);
  const int t = lane & ((1 << logT) - 1);
  const int lig = (lane >> logT) & (G - 1);
  const int sub = lane >> (logT + LG);
  const int per_wave = kWave >> (logT + LG);  // pairs one wave covers side by side
  kptr<ClassRec> classes = kconst(P.classes);
  const bool uni = S.cls_fixed >= 0;
  ProdParams pp_uni{};
  if constexpr (KIND == KIND_PROD1 || KIND == KIND_PROD2) {
    if (uni) pp_uni = prod_params(classes, S.cls_fixed);
  }
  // Software pipeline: the next chunk of U * per_wave constraints is claimed
  // and its literal codes are loaded before the current chunk is evaluated, so
  // the load latency overlaps the LDS and ALU work of the current chunk.
  auto claim = [&]() {
    int b = 0;
    if (lane == 0) b = atomicAdd(ctr, U * per_wave);
    return __builtin_amdgcn_readfirstlane(b);
  };
  auto fetch = [&](int b, FetchedU<J, U>& f) {
#pragma unroll
    for (int u = 0; u < U; ++u) fetch_pair<J, KMAX>(P, S, b + u * per_wave + sub, lig, f.p[u]);
  };
  int base = claim();
  FetchedU<J, U> cur;
  fetch(base, cur);
  while (base < S.c_count) {
    const int nbase = claim();
    FetchedU<J, U> nxt;
    fetch(nbase, nxt);
    // A chunk (aligned, fixed pairs per lane, fixed order) sums its objective
    // terms in FP32 and adds one exact fixed-point term: the result does not
    // depend on which wave claimed the chunk.
    float fchunk = 0.f;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b_u = base + u * per_wave;
      if (u > 0 && b_u >= S.c_count) break;  // wave-uniform: the rest of the chunk is past the segment
      const Fetched<J>& fp = cur.p[u];
      const bool valid = b_u + sub < S.c_count;
      // constraints are sorted by class inside a segment, so most chunks hold
      // one class: then its parameters are read once per wave with scalar loads
      const int c0 = __builtin_amdgcn_readfirstlane(fp.cls);  // lane 0 holds a valid pair
      const bool chunk_uni = uni || !__any(valid && fp.cls != c0);
      auto eval_pair = [&](auto& sink, const Fetched<J>& f) {
        if constexpr (KIND == KIND_DFT || (KIND == KIND_PMF && KMAX > 8)) {
          // lanes take turns by class (the first remaining lane's class each
          // round; one round for a class-uniform chunk), so the class record,
          // node table and window coefficients are always read with scalar loads
          for (;;) {
            const int cc = __builtin_amdgcn_readfirstlane(f.cls);
            if (f.cls == cc) {
              if constexpr (KIND == KIND_DFT) {
                kptr<ClassRec> cr = kconst(P.classes);
                dft_pair<KMAX, G>(P, cr[cc].n_nodes, cc, f, lig, t, logT, xs, sink, fchunk, gsc, fsc);
              } else if constexpr (G == 8) {
                pmfg8_pair<KMAX>(P, cc, f, lig, t, logT, xs, sink, fchunk, gsc, fsc);
              } else {
                pmfg_pair<KMAX, G>(P, cc, f, lig, t, logT, xs, sink, fchunk, gsc, fsc);
              }
              break;
            }
          }
        } else if constexpr (KIND == KIND_PMF) {
          // window width of the segment (uniform): 2, 3 or 4 counts
          const int cls = chunk_uni ? c0 : f.cls;
          if (S.m_max <= 2) {
            pmf_pair<KMAX, 2>(P, cls, f, t, logT, xs, sink, fchunk, gsc, fsc);
          } else if (S.m_max == 3) {
            pmf_pair<KMAX, 3>(P, cls, f, t, logT, xs, sink, fchunk, gsc, fsc);
          } else {
            pmf_pair<KMAX, 4>(P, cls, f, t, logT, xs, sink, fchunk, gsc, fsc);
          }
        } else {
          const ProdParams pp = uni ? pp_uni : prod_params(classes, chunk_uni ? c0 : f.cls);
          prod_pair<KIND == KIND_PROD2 ? 2 : 1, KMAX, G>(f, lig, t, logT, P.n, xs, sink, fchunk, gsc, fsc, pp);
        }
      };
      if constexpr (ST) {
        // unweighted terms: weight 1 and scale 1 (gsc = 1 in this kernel)
        float sq = 0.f;
        if (valid) {
          Fetched<J> f1 = fp;
          f1.w = 1.f;
          SquareSink sk{0.f, P.n};
          eval_pair(sk, f1);
          sq = sk.acc;
        }
        for (int o = 1 << logT; o < (G << logT); o <<= 1) sq += __shfl_xor(sq, o);  // the pair's G lanes
        if (valid && lig == 0) atomicAdd(&so.acc[S.c_begin + b_u + sub], (unsigned long long)fixed_term(sq * so.scale));
      } else {
        if (valid) {
          GradSink<AT> sk{gs};
          eval_pair(sk, fp);
        }
      }
    }
    facc.own += fixed_term(fchunk);
    cur = nxt;
    base = nbase;
  }
}

#define PCLS_BUCKET_CASES(KIND, X) \
  X(KIND, 0, 1)                    \
  X(KIND, 1, 2)                    \
  X(KIND, 2, 3)                    \
  X(KIND, 3, 4)                    \
  X(KIND, 4, 5)                    \
  X(KIND, 5, 6)                    \
  X(KIND, 6, 7)                    \
  X(KIND, 7, 8)                    \
  X(KIND, 8, 12)                   \
  X(KIND, 9, 16)                   \
  X(KIND, 10, 24)                  \
  X(KIND, 11, 32)                  \
  X(KIND, 12, 48)                  \
  X(KIND, 13, 64)                  \
  X(KIND, 14, 96)                  \
  X(KIND, 15, 128)                 \
  X(KIND, 16, 192)                 \
  X(KIND, 17, 256)

#define PCLS_SHORT_BUCKET_CASES(KIND, X) \
  X(KIND, 0, 1)                          \
  X(KIND, 1, 2)                          \
  X(KIND, 2, 3)                          \
  X(KIND, 3, 4)                          \
  X(KIND, 4, 5)                          \
  X(KIND, 5, 6)                          \
  X(KIND, 6, 7)                          \
  X(KIND, 7, 8)

#define PCLS_PMF_BUCKET_CASES(KIND, X) \
  PCLS_SHORT_BUCKET_CASES(KIND, X)       \
  X(KIND, 8, 12)                         \
  X(KIND, 9, 16)                         \
  X(KIND, 10, 24)                        \
  X(KIND, 11, 32)                        \
  X(KIND, 12, 48)

#define PCLS_CASE(KIND, B, KMAX)                                                                    \
  case (KIND)*kNumBuckets + (B):                                                                    \
    if constexpr ((B) <= MAXB) run_segment<KIND, KMAX, MAXB, AT, ST>(P, S, xs, gs, facc, gsc, fsc, tid, logT, ctr, so); \
    break;

template <int MAXB, class AT, bool ST = false>
__device__ __forceinline__ void run_any_segment(const ProblemDev& P, const Segment& S, const float* xs, AT* gs,
                                                ObjAcc& facc, float gsc, float fsc, int tid, int logT,
                                                int* ctr, StatsOut so = {}) {
  switch (S.kind * kNumBuckets + S.bucket) {
    PCLS_BUCKET_CASES(KIND_PROD1, PCLS_CASE)
    PCLS_BUCKET_CASES(KIND_PROD2, PCLS_CASE)
    PCLS_BUCKET_CASES(KIND_DFT, PCLS_CASE)
    PCLS_PMF_BUCKET_CASES(KIND_PMF, PCLS_CASE)
    default:
      break;
  }
}

// Arguments of one resident tile: restarts [r0, r0 + 2^logT) of one problem.
struct TileArgs {
  float* X;          // [n][ldx] state
  int R, ldx, r0, logT;
  float lr;
  int n_steps;
  float* trace;      // [n_steps][R] or NULL
  float* obj_out;    // evaluate mode: [R]; NULL = step mode
  float* g_out;      // evaluate mode: [n][ldx] or NULL
  float gsc, ginv;   // gradient fixed-point scale 2^S and 2^-S
  float fsc, finv;   // objective fixed-point scale
  const int8_t* fixed;  // [n] or NULL: 0 free, -1 / +1 variable held at that corner value
  float tol;            // > 0: convergence test max_v |dx| < tol per restart
  int* iters;           // [R] or NULL: steps until convergence (n_steps if never)
};

// In the variants for short constraints, whose steps are short enough for the
// end-of-step reduction to matter, objective partial sums leave the lanes in
// two stages without wave shuffles (those go through the LDS crossbar, which
// all waves of the tile would contend for at once).  Within each 16-lane
// row, DPP row shifts (VALU only, no LDS traffic) add up the lanes of equal
// index mod P, so the top P lanes of the row hold the row's sums (P >= 16:
// nothing to fold).  Those lanes then add into 64-bit LDS slots, slot
// r * P + (lane mod P) for row r (P >= 16: slot = lane): at most 4 slots per
// residue, all distinct within a wave.  Integer sums are exact in any order.
template <int D>
__device__ __forceinline__ unsigned long long add_row_shr(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, 0x110 + D, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), 0x110 + D, 0xf, 0xf, true);
  return v + (((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ unsigned long long row_fold(unsigned long long v, int P) {
  if (P <= 1) v = add_row_shr<1>(v);
  if (P <= 2) v = add_row_shr<2>(v);
  if (P <= 4) v = add_row_shr<4>(v);
  if (P <= 8) v = add_row_shr<8>(v);
  return v;
}
// slot of this lane's folded sum, or -1 (lanes whose row sum sits elsewhere)
__device__ __forceinline__ int fold_slot(int lane, int P) {
  if (P >= 16) return lane;
  const int c = lane & 15;
  return c >= 16 - P ? (lane >> 4) * P + (c - (16 - P)) : -1;
}
// sum and clear the slots of residue q (slots q + r P, r < min(4, 64 / P))
__device__ __forceinline__ unsigned long long take_slots(unsigned long long* sl, int q, int P) {
  const int nper = P >= 16 ? kWave / P : 4;
  unsigned long long a[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (r < nper) a[r] = sl[q + r * P];
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (r < nper) sl[q + r * P] = 0ull;
  return (a[0] + a[1]) + (a[2] + a[3]);
}

// All n_steps steps of one tile with its state in LDS.
// LDS: x[n][T] float | g[n][T] fixed point | two slot sets for the objective
//      (64-bit fixed point; per set 64 slots, and 2 x 64 more for the even and
//      odd restarts of two-restart lanes when T >= 2; the long-constraint
//      variants use slot t of set 0 for restart t) |
//      one work counter per segment | per restart: converged flag, max |dx|.
template <int MAXB, class AT>
__device__ __forceinline__ void resident_tile(const ProblemDev& P, const TileArgs& A, unsigned long long* lds_raw) {
  const int logT = A.logT;
  const int T = 1 << logT;
  const int NT = P.n << logT;                 // state elements stepped
  const int NR = (P.n + P.n_pad) << logT;     // with the pad rows
  float* xs = reinterpret_cast<float*>(lds_raw);
  AT* gs = reinterpret_cast<AT*>(reinterpret_cast<char*>(lds_raw) + ((size_t)NR * 4 + 15) / 16 * 16);
  unsigned long long* Fl =
      reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(gs) + ((size_t)NR * sizeof(AT) + 7) / 8 * 8);
  const int n_fl = logT >= 1 ? 3 * kWave : kWave;  // slots per set; two sets
  int* ctr = reinterpret_cast<int*>(Fl + 2 * n_fl);
  int* conv = ctr + kMaxSegments;
  unsigned int* dxmax = reinterpret_cast<unsigned int*>(conv + T);
  const int tid = threadIdx.x, nth = blockDim.x;
  const int r0 = A.r0, ldx = A.ldx;
  const int t = tid & (T - 1);
  const bool eval = A.obj_out != nullptr;
  const int n_seg = P.n_segments;

  for (int i = tid; i < NT; i += nth) {
    const int v = i >> logT, tt = i & (T - 1);
    float x = A.X[(size_t)v * ldx + r0 + tt];
    if (A.fixed && A.fixed[v] != 0) x = (float)A.fixed[v];
    xs[i] = x;
    gs[i] = 0;
  }
  for (int i = NT + tid; i < NR; i += nth) {  // pad rows: x = +1, never stepped
    xs[i] = 1.f;
    gs[i] = 0;
  }
  for (int i = tid; i < 2 * n_fl; i += nth) Fl[i] = 0ull;
  if (tid < T) {
    conv[tid] = 0;
    dxmax[tid] = 0u;
  }
  if (tid < n_seg) ctr[tid] = 0;
  __syncthreads();
  float F_last = 0.f;  // threads tid < T: last evaluated objective of restart r0 + tid

  // The objective of step s goes through slot set s mod 2.  deposit: every wave
  // adds its lanes' partial sums; finalize: thread t < T, once every deposit of
  // that step has landed, sums and clears restart t's slots and writes F.
  auto set_of = [&](int step) { return Fl + (step & 1) * n_fl; };
  auto deposit = [&](const ObjAcc& fa, unsigned long long* sl) {
    if constexpr (MAXB <= kMaxbShort) {
      // restart of a lane's own terms: lane mod T; of its two-restart terms:
      // 2 (lane mod T/2) (even) and 2 (lane mod T/2) + 1 (odd).
      // (opaque lane index: slot addresses are recomputed here each step instead
      // of being kept live through the segment loops)
      int l = tid & (kWave - 1);
      asm volatile("" : "+v"(l));
      const unsigned long long vo = row_fold((unsigned long long)fa.own, T);
      const int so = fold_slot(l, T);
      if (so >= 0) atomicAdd(&sl[so], vo);
      if (logT >= 1) {
        const unsigned long long ve = row_fold((unsigned long long)fa.even, T >> 1);
        const unsigned long long vd = row_fold((unsigned long long)fa.odd, T >> 1);
        const int s2 = fold_slot(l, T >> 1);
        if (s2 >= 0) {
          atomicAdd(&sl[kWave + s2], ve);
          atomicAdd(&sl[2 * kWave + s2], vd);
        }
      }
    } else {
      // variants for long constraints: a step's work dwarfs this reduction, and
      // the shuffle form leaves the register allocation of their long loops
      // unchanged (the row fold above made them spill more)
      unsigned long long v = (unsigned long long)fa.own;
      for (int o = T; o < kWave; o <<= 1) v += __shfl_xor(v, o);
      if ((tid & (kWave - 1)) < T) atomicAdd(&sl[t], v);
    }
  };
  auto finalize = [&](int step, unsigned long long* sl) {
    // each slot has one reader, which clears it for the step after next
    unsigned long long acc;
    if constexpr (MAXB <= kMaxbShort) {
      int q = t;
      asm volatile("" : "+v"(q));
      acc = take_slots(sl, q, T);
      if (logT >= 1) acc += take_slots(sl + ((q & 1) ? 2 * kWave : kWave), q >> 1, T >> 1);
    } else {
      acc = sl[t];
      sl[t] = 0ull;
    }
    const float F = FixedAcc<unsigned long long>::value_exact(acc, A.finv) + P.f_const;
    const int r = r0 + tid;
    F_last = F;
    if (r < A.R) {
      if (A.trace) A.trace[(size_t)step * A.R + r] = F;
      if (eval) A.obj_out[r] = F;
    }
  };
  // Short-constraint variants take the objective of step s off the critical
  // path: its deposits and step s-1's finalize run at the start of step s + 1,
  // where the dynamic work claims absorb them (a wave that spends time there
  // claims fewer chunks).  Long-constraint variants reduce within the step.
  constexpr bool kDefer = MAXB <= kMaxbShort;
  ObjAcc prev{0, 0, 0};
  int done = A.n_steps;  // steps taken (fewer once every restart has converged)

  for (int s = 0; s < A.n_steps; ++s) {
    if constexpr (kDefer) {
      if (s > 0) {
        deposit(prev, set_of(s - 1));
        if (s > 1 && tid < T) finalize(s - 2, set_of(s - 2));
      }
    }
    ObjAcc facc{0, 0, 0};
    kptr<Segment> segs = kconst(P.segments);
    for (int sg = 0; sg < n_seg; ++sg) {
      const Segment S{segs[sg].kind,    segs[sg].bucket, segs[sg].c_begin,   segs[sg].c_count,
                      segs[sg].lit_base, segs[sg].k_fixed, segs[sg].cls_fixed, segs[sg].m_max};
      run_any_segment<MAXB>(P, S, xs, gs, facc, A.gsc, A.fsc, tid, logT, ctr + sg);
    }
    if constexpr (!kDefer) deposit(facc, set_of(0));
    __syncthreads();
    if (tid < n_seg) ctr[tid] = 0;  // every wave has left the segment loops
    if constexpr (!kDefer) {
      if (tid < T) finalize(s, set_of(0));
    } else {
      prev = facc;
    }
    if (eval) {
      if (A.g_out) {
        for (int i = tid; i < NT; i += nth) {
          const int v = i >> logT, tt = i & (T - 1);
          A.g_out[(size_t)v * ldx + r0 + tt] = FixedAcc<AT>::value(gs[i], A.ginv, P.occ[v]);
        }
      }
    } else if (sizeof(AT) == 4 && A.tol <= 0.f && !A.fixed && (NT & 3) == 0) {
      // plain step, 32-bit accumulator: four elements per 16-byte LDS access
      // (same arithmetic per element as the general loop below)
      const float lr = A.lr, ginv = A.ginv;
      float4* x4 = reinterpret_cast<float4*>(xs);
      uint4* g4 = reinterpret_cast<uint4*>(gs);
      for (int i = tid; i < (NT >> 2); i += nth) {
        float4 x = x4[i];
        const uint4 g = g4[i];
        x.x = fminf(1.f, fmaxf(-1.f, fmaf(-lr, (float)(int)g.x * ginv, x.x)));
        x.y = fminf(1.f, fmaxf(-1.f, fmaf(-lr, (float)(int)g.y * ginv, x.y)));
        x.z = fminf(1.f, fmaxf(-1.f, fmaf(-lr, (float)(int)g.z * ginv, x.z)));
        x.w = fminf(1.f, fmaxf(-1.f, fmaf(-lr, (float)(int)g.w * ginv, x.w)));
        x4[i] = x;
        g4[i] = make_uint4(0u, 0u, 0u, 0u);
      }
    } else {
      const float lr = A.lr;
      float dmax = 0.f;  // this thread's elements all belong to restart t (nth is a multiple of T)
      for (int i = tid; i < NT; i += nth) {
        const int v = i >> logT;
        float xn = fmaf(-lr, FixedAcc<AT>::value(gs[i], A.ginv, P.occ[v]), xs[i]);
        xn = fminf(1.f, fmaxf(-1.f, xn));
        if (A.fixed && A.fixed[v] != 0) xn = (float)A.fixed[v];
        dmax = fmaxf(dmax, fabsf(xn - xs[i]));
        xs[i] = xn;
        gs[i] = 0;
      }
      if (A.tol > 0.f) {
        for (int o = T; o < kWave; o <<= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, o));
        if ((tid & (kWave - 1)) < T) atomicMax(&dxmax[t], __float_as_uint(dmax));  // dmax >= 0: bits are monotone
      }
    }
    __syncthreads();
    if (!eval && A.tol > 0.f) {
      // convergence: a tile stops once every restart in it has converged
      if (tid < T) {
        const int r = r0 + tid;
        if (!conv[tid] && __uint_as_float(dxmax[tid]) < A.tol) {
          conv[tid] = 1;
          if (A.iters && r < A.R) A.iters[r] = s + 1;
        }
        dxmax[tid] = 0u;
      }
      __syncthreads();
      int all = 1;
      for (int q = 0; q < T; ++q) all &= conv[q];
      __syncthreads();  // flags read before the next step may change them
      if (all) {
        done = s + 1;
        break;
      }
    }
  }
  if constexpr (kDefer) {
    if (done > 0) {
      deposit(prev, set_of(done - 1));
      if (done > 1 && tid < T) finalize(done - 2, set_of(done - 2));
      __syncthreads();
      if (tid < T) finalize(done - 1, set_of(done - 1));
    }
  }
  // a tile that stopped early repeats its last objective for the remaining steps
  if (tid < T && A.trace && r0 + tid < A.R)
    for (int q = done; q < A.n_steps; ++q) A.trace[(size_t)q * A.R + r0 + tid] = F_last;
  if (!eval && A.tol > 0.f && A.iters && tid < T && r0 + tid < A.R && !conv[tid]) A.iters[r0 + tid] = A.n_steps;
  if (!eval) {
    for (int i = tid; i < NT; i += nth) {
      const int v = i >> logT, tt = i & (T - 1);
      A.X[(size_t)v * ldx + r0 + tt] = xs[i];
    }
  }
}

// One workgroup per tile of T = 2^logT restarts; all n_steps steps in LDS.
// Evaluate mode (obj_out != NULL): one evaluation, writes F and optionally G.
// Variants by the largest length bucket they handle (a kernel's register
// allocation covers its longest code path, so short-constraint problems run a
// variant with fewer registers and more waves per SIMD) and by the width of the
// fixed-point gradient accumulator (64-bit, or 32-bit where LDS is short).
template <int MAXB, class AT>
__global__ void __launch_bounds__(1024) tile_kernel(ProblemDev P, TileArgs A) {
  extern __shared__ __attribute__((aligned(16))) unsigned long long lds_raw[];  // 16 B: vector LDS accesses
  A.r0 = blockIdx.x << A.logT;
  resident_tile<MAXB, AT>(P, A, lds_raw);
}

// ---------------------------------------------------- constraint statistics
// One workgroup per restart evaluates every constraint once and adds, per
// constraint, the sum over its literals of (dFE_c/dy_i)^2 (unweighted) into a
// 64-bit fixed-point accumulator: exact integer sums, so the result does not
// depend on the order in which restarts or waves arrive.
template <int MAXB>
__global__ void __launch_bounds__(1024) stats_kernel(ProblemDev P, const float* __restrict__ X, int ldx,
                                                     StatsOut so) {
  extern __shared__ __attribute__((aligned(16))) unsigned long long lds_raw[];  // 16 B: vector LDS accesses
  float* xs = reinterpret_cast<float*>(lds_raw);
  int* ctr = reinterpret_cast<int*>(xs + ((P.n + P.n_pad + 1) & ~1));
  const int r = blockIdx.x;
  for (int i = threadIdx.x; i < P.n + P.n_pad; i += blockDim.x) xs[i] = i < P.n ? X[(size_t)i * ldx + r] : 1.f;
  if ((int)threadIdx.x < P.n_segments) ctr[threadIdx.x] = 0;
  __syncthreads();
  ObjAcc facc{0, 0, 0};
  kptr<Segment> segs = kconst(P.segments);
  for (int sg = 0; sg < P.n_segments; ++sg) {
    const Segment S{segs[sg].kind,    segs[sg].bucket, segs[sg].c_begin,   segs[sg].c_count,
                    segs[sg].lit_base, segs[sg].k_fixed, segs[sg].cls_fixed, segs[sg].m_max};
    run_any_segment<MAXB, unsigned int, true>(P, S, xs, nullptr, facc, 1.f, 0.f, (int)threadIdx.x, 0, ctr + sg, so);
  }
}

// acc (planned order, scale 2^s) -> out[caller's constraint index]
__global__ void stats_finish_kernel(const unsigned long long* __restrict__ acc, const int32_t* __restrict__ perm,
                                    int m, double inv, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[perm[i]] = (float)((double)(long long)acc[i] * inv);
}

// ------------------------------------------------------------ batched engine
// Many problems (instances) and their restart tiles in one persistent launch.
// Work items (instance, first restart, tile size) are claimed from a counter in
// order of decreasing cost; a workgroup keeps claiming until the list is empty.

struct BatchInst {
  ProblemDev P;
  float* X;
  float* trace;
  int R, ldx;
  float gsc, ginv, fsc, finv;
};

struct BatchItem {
  int inst, r0, logT, pad;
};

__device__ __forceinline__ ProblemDev load_problem(kptr<BatchInst> bi) {
  ProblemDev P;
  P.n = bi->P.n;
  P.n_pad = bi->P.n_pad;
  P.m = bi->P.m;
  P.L = bi->P.L;
  P.n_segments = bi->P.n_segments;
  P.n_classes = bi->P.n_classes;
  P.f_const = bi->P.f_const;
  P.segments = bi->P.segments;
  P.classes = bi->P.classes;
  P.nodes = bi->P.nodes;
  P.sp = bi->P.sp;
  P.litT = bi->P.litT;
  P.c_k = bi->P.c_k;
  P.c_cls = bi->P.c_cls;
  P.c_w = bi->P.c_w;
  P.row_ptr = bi->P.row_ptr;
  P.lit = bi->P.lit;
  P.unit_weights = bi->P.unit_weights;
  P.max_k = bi->P.max_k;
  P.occ = bi->P.occ;
  return P;
}

template <int MAXB, class AT>
__global__ void __launch_bounds__(1024) batch_kernel(const BatchInst* __restrict__ insts,
                                                     const BatchItem* __restrict__ items, int n_items,
                                                     unsigned int* __restrict__ counter, float lr, int n_steps,
                                                     int claim_off) {
  extern __shared__ __attribute__((aligned(16))) unsigned long long lds_raw[];  // 16 B: vector LDS accesses
  // the claimed item's word sits after the largest tile (no static LDS)
  int* claimed = reinterpret_cast<int*>(reinterpret_cast<char*>(lds_raw) + claim_off);
  for (;;) {
    if (threadIdx.x == 0) *claimed = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int it = *claimed;
    __syncthreads();
    if (it >= n_items) break;  // every workgroup reaches this once the list is drained
    kptr<BatchItem> W = kconst(items) + it;
    kptr<BatchInst> B = kconst(insts) + W->inst;
    const ProblemDev P = load_problem(B);
    TileArgs A;
    A.X = B->X;
    A.R = B->R;
    A.ldx = B->ldx;
    A.r0 = W->r0;
    A.logT = W->logT;
    A.lr = lr;
    A.n_steps = n_steps;
    A.trace = B->trace;
    A.obj_out = nullptr;
    A.g_out = nullptr;
    A.gsc = B->gsc;
    A.ginv = B->ginv;
    A.fsc = B->fsc;
    A.finv = B->finv;
    A.fixed = nullptr;
    A.tol = 0.f;
    A.iters = nullptr;
    resident_tile<MAXB, AT>(P, A, lds_raw);
    __syncthreads();
  }
}

__global__ void fill_u32_kernel(unsigned int* p, unsigned int v, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// ------------------------------------------------------------------- init

__device__ __forceinline__ uint32_t philox_first_word(uint32_t c0, uint32_t c1, uint32_t k0, uint32_t k1) {
  uint32_t c2 = 0u, c3 = 0u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c1 = lo1;
    c3 = lo0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c0;
}

// mask != NULL: only restarts r < R with mask[r] != 0 are written.
__global__ void init_kernel(float* __restrict__ X, int n, int R, int ldx, uint32_t k0, uint32_t k1,
                            const uint8_t* __restrict__ mask) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (r >= ldx || v >= n) return;
  if (mask && (r >= R || mask[r] == 0)) return;
  float x = 0.f;
  if (r < R) {
    const uint32_t o = philox_first_word((uint32_t)r, (uint32_t)v, k0, k1);
    x = (float)((int32_t)(o >> 8) - 8388608) * (1.0f / 8388608.0f);
  }
  X[(size_t)v * ldx + r] = x;
}

// ---------------------------------------------------------------- extract

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// lane = restart; each block row covers a chunk of constraints
__global__ void extract_count_kernel(ProblemDev P, const float* __restrict__ X, int R, int ldx,
                                     int32_t* __restrict__ unsat, int chunk) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int c0 = blockIdx.y * chunk;
  const int c1 = min(P.m, c0 + chunk);
  if (r >= R) return;
  int cnt = 0;
  for (int c = c0; c < c1; ++c) {
    const int b = P.row_ptr[c], e = P.row_ptr[c + 1];
    int ntrue = 0;
    for (int i = b; i < e; ++i) {
      const int code = P.lit[i];
      const bool var_true = X[(size_t)(code >> 1) * ldx + r] < 0.f;
      ntrue += (var_true != (bool)(code & 1)) ? 1 : 0;
    }
    const int sp_off = kconst(P.classes)[P.c_cls[c]].sp_off;
    cnt += P.sp[sp_off + ntrue] > 0 ? 1 : 0;
  }
  if (cnt) atomicAdd(&unsat[r], cnt);
}

// 64 x 64 tile transpose: X[v][r] -> assign[r][v]
__global__ void extract_assign_kernel(const float* __restrict__ X, int n, int R, int ldx, int8_t* __restrict__ assign) {
  __shared__ int8_t tile[64][65];
  const int r0 = blockIdx.x * 64, v0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 256 threads: 4 rows per pass
  for (int q = ty; q < 64; q += 4) {
    const int v = v0 + q, r = r0 + tx;
    int8_t z = 1;
    if (v < n && r < R) z = X[(size_t)v * ldx + r] < 0.f ? (int8_t)-1 : (int8_t)1;
    tile[q][tx] = z;
  }
  __syncthreads();
  for (int q = ty; q < 64; q += 4) {
    const int r = r0 + q, v = v0 + tx;
    if (r < R && v < n) assign[(size_t)r * n + v] = tile[tx][q];
  }
}

__global__ void extract_best_kernel(const int32_t* __restrict__ unsat, int R, int32_t* __restrict__ best) {
  __shared__ unsigned long long red[1024];
  unsigned long long key = ~0ull;
  for (int r = threadIdx.x; r < R; r += blockDim.x) {
    const unsigned long long kk = ((unsigned long long)(uint32_t)unsat[r] << 32) | (uint32_t)r;
    key = kk < key ? kk : key;
  }
  red[threadIdx.x] = key;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const unsigned long long o = red[threadIdx.x + s];
      if (o < red[threadIdx.x]) red[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) best[0] = R > 0 ? (int32_t)(red[0] & 0xffffffffu) : -1;
}

// ------------------------------------------------------------------ host side

int32_t hip_fail(hipError_t e, const char* what) {
  (void)hipGetLastError();  // clear the runtime's sticky error so later callers do not inherit it
  return set_error(PCLS_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define PCLS_HIP(call, what)                 \
  do {                                       \
    hipError_t _e = (call);                  \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

int round_up64(int R) { return (R + 63) / 64 * 64; }

struct DeviceLimits {
  int lds_max = 0;
  int n_cu = 0;
  bool lds_attr_set = false;
};

std::mutex g_dev_mu;
DeviceLimits g_dev[64];

// The literal gathers address x by its LDS byte offset alone, which holds only
// while a kernel's dynamic LDS starts at address 0: no static LDS.
hipError_t check_no_static_lds(const void* f) {
  hipFuncAttributes a{};
  hipError_t e = hipFuncGetAttributes(&a, f);
  if (e != hipSuccess) return e;
  return a.sharedSizeBytes == 0 ? hipSuccess : hipErrorInvalidKernelFile;
}

int32_t device_limits(DeviceLimits& out) {
  int dev = 0;
  PCLS_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) return set_error(PCLS_E_HIP, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_dev_mu);
  DeviceLimits& d = g_dev[dev];
  if (d.lds_max == 0) {
    int v = 0;
    PCLS_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "hipDeviceGetAttribute");
    d.lds_max = v;
    PCLS_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
    d.n_cu = v;
  }
  if (!d.lds_attr_set) {
    const void* variants[] = {(const void*)tile_kernel<kMaxbShort, unsigned long long>,
                              (const void*)tile_kernel<kMaxbMid, unsigned long long>,
                              (const void*)tile_kernel<kMaxbAll, unsigned long long>,
                              (const void*)tile_kernel<kMaxbShort, unsigned int>,
                              (const void*)tile_kernel<kMaxbMid, unsigned int>,
                              (const void*)tile_kernel<kMaxbAll, unsigned int>,
                              (const void*)stats_kernel<kMaxbShort>,
                              (const void*)stats_kernel<kMaxbMid>,
                              (const void*)stats_kernel<kMaxbAll>};
    for (const void* f : variants) {
      PCLS_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, d.lds_max), "hipFuncSetAttribute");
      PCLS_HIP(check_no_static_lds(f), "kernel attributes");
    }
    d.lds_attr_set = true;
  }
  out = d;
  return PCLS_OK;
}

// LDS of one workgroup: x[n][T] float, g[n][T] fixed point (4 or 8 bytes),
// F[T] 64-bit, each region 8-byte aligned.
size_t tile_lds_bytes(int rows, int T, int acc_bytes) {
  const size_t nt = (size_t)rows * T;
  const size_t slots = 2 * (T >= 2 ? 3 : 1) * (size_t)kWave * 8;  // two sets of objective slots
  return (nt * 4 + 15) / 16 * 16 + (nt * acc_bytes + 7) / 8 * 8 + slots + 4 * kMaxSegments + (size_t)T * 8;
}

// rows of the on-chip state: the variables and the pad rows
int state_rows(const pcls_problem* p) { return p->n + p->n_pad; }

struct Launch {
  int logT;
  int block;
  size_t lds;
  bool acc64;
};

// Restarts per workgroup: largest power of two whose state fits in LDS, at
// most 64 / G_max (a lane group must stay inside one wave), and small enough
// to give every compute unit at least two tiles when R allows it.  The 64-bit
// gradient accumulator is used whenever its tile fits, else the 32-bit one.
// Automatic accumulator width.  A 32-bit accumulator whose quantum is at most
// 2^-24 (the FP32 unit roundoff at 1) adds no more error per term than the FP32
// arithmetic that produced the term, and halves the LDS atomic traffic and the
// state footprint; otherwise 64 bits are used wherever the state fits.
constexpr int kAcc32MinScale = 24;

bool auto_acc64(const pcls_problem* p, size_t cap) {
  if (p->acc_bits == 64) return true;
  if (p->acc_bits == 32) return false;
  if (p->s_g32 >= kAcc32MinScale) return false;
  return tile_lds_bytes(state_rows(p), std::max(1, p->tile_restarts), 8) <= cap;
}

int32_t choose_launch(const pcls_problem* p, int R, Launch& L) {
  DeviceLimits lim;
  int32_t st = device_limits(lim);
  if (st != PCLS_OK) return st;
  const int R_pad = round_up64(R);
  const int tmax_group = kWave / std::max(1, p->max_group);
  const size_t cap = (size_t)lim.lds_max;
  const bool acc64 = auto_acc64(p, cap);
  if (!acc64 && p->s_g32 < 8)
    return set_error(PCLS_E_UNSUPPORTED, "state of %d variables does not fit on chip with a 64-bit accumulator and "
                     "weights are too large for a 32-bit one", p->n);
  const int ab = acc64 ? 8 : 4;
  int T;
  if (p->tile_restarts > 0) {
    T = p->tile_restarts;
  } else {
    // the widest tile that still gives every CU a tile: more restarts per tile
    // share each literal-code fetch and spread a wave's LDS accesses over
    // fewer variables (fewer bank conflicts)
    T = 1;
    const int want_tiles = std::max(1, lim.n_cu);
    while (T * 2 <= tmax_group && tile_lds_bytes(state_rows(p), T * 2, ab) <= cap && R_pad / (T * 2) >= want_tiles) T *= 2;
  }
  if (T < 1 || T > 64 || (T & (T - 1)))
    return set_error(PCLS_E_INVALID, "tile_restarts %d must be a power of two in [1, 64]", T);
  if (T > tmax_group)
    return set_error(PCLS_E_UNSUPPORTED, "tile_restarts %d too large for constraints of %d literals", T, p->max_k);
  const size_t lds = tile_lds_bytes(state_rows(p), T, ab);
  if (lds > cap)
    return set_error(PCLS_E_UNSUPPORTED,
                     "state of %d variables x %d restarts needs %zu bytes of LDS (device limit %d)", p->n, T, lds,
                     lim.lds_max);
  int block = p->block_threads;
  if (block <= 0) block = (lds > cap / 2 || R_pad / T <= lim.n_cu) ? 1024 : 512;
  if (block != 256 && block != 512 && block != 1024)
    return set_error(PCLS_E_INVALID, "block_threads %d must be 256, 512 or 1024", block);
  L.logT = 0;
  while ((1 << L.logT) < T) ++L.logT;
  L.block = block;
  L.lds = lds;
  L.acc64 = acc64;
  return PCLS_OK;
}

int32_t check_bound(const pcls_problem* p) {
  if (!p) return set_error(PCLS_E_INVALID, "problem handle is NULL");
  if (!p->d_ws) return set_error(PCLS_E_WORKSPACE, "problem has no device workspace (call pcls_upload)");
  return PCLS_OK;
}

int32_t launch_tile(const pcls_problem* p, int R, float* d_x, float lr, int n_steps, float* trace, float* obj,
                    float* grad, hipStream_t stream, const pcls_step_options* opt = nullptr) {
  Launch L;
  int32_t st = choose_launch(p, R, L);
  if (st != PCLS_OK) return st;
  const int R_pad = round_up64(R);
  const int tiles = (R + (1 << L.logT) - 1) >> L.logT;  // padding-only tiles are skipped
  const int sg = L.acc64 ? p->s_g64 : p->s_g32;
  TileArgs A;
  A.X = d_x;
  A.R = R;
  A.ldx = R_pad;
  A.r0 = 0;
  A.logT = L.logT;
  A.lr = lr;
  A.n_steps = n_steps;
  A.trace = trace;
  A.obj_out = obj;
  A.g_out = grad;
  A.gsc = std::ldexp(1.0f, sg);
  A.ginv = std::ldexp(1.0f, -sg);
  A.fsc = std::ldexp(1.0f, p->s_f);
  A.finv = std::ldexp(1.0f, -p->s_f);
  A.fixed = opt ? opt->d_fixed : nullptr;
  A.tol = opt ? opt->tol : 0.f;
  A.iters = opt ? opt->d_iters : nullptr;
  void (*kern)(ProblemDev, TileArgs);
  if (L.acc64) {
    kern = p->max_bucket <= kMaxbShort ? tile_kernel<kMaxbShort, unsigned long long>
           : p->max_bucket <= kMaxbMid ? tile_kernel<kMaxbMid, unsigned long long>
                                       : tile_kernel<kMaxbAll, unsigned long long>;
  } else {
    kern = p->max_bucket <= kMaxbShort ? tile_kernel<kMaxbShort, unsigned int>
           : p->max_bucket <= kMaxbMid ? tile_kernel<kMaxbMid, unsigned int>
                                       : tile_kernel<kMaxbAll, unsigned int>;
  }
  hipLaunchKernelGGL(kern, dim3(tiles), dim3(L.block), L.lds, stream, p->dev, A);
  PCLS_HIP(hipGetLastError(), "tile_kernel launch");
  return PCLS_OK;
}

// ------------------------------------------------------------ batch (host)

struct BatchState {
  std::vector<const pcls_problem*> probs;
  std::vector<int> R;
  std::vector<float*> x, trace;
  pcls_batch_config cfg{};
  bool acc64 = true;
  int maxb = 0;
  int n_items = 0;
  size_t lds = 0;   // dynamic LDS of the persistent launch
  int grid = 0;
  void* d_ws = nullptr;
  size_t ws_bytes = 0;
  size_t off_inst = 0, off_items = 0, off_counter = 0;
  std::vector<BatchInst> inst;
  std::vector<BatchItem> items;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~BatchState() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

size_t batch_ws_bytes(int count, size_t max_items) {
  size_t off = 0;
  auto place = [&](size_t b) {
    off = (off + 255) / 256 * 256;
    size_t at = off;
    off += b;
    return at;
  };
  place(sizeof(BatchInst) * (size_t)count);
  place(sizeof(BatchItem) * max_items);
  place(256);
  return (off + 255) / 256 * 256;
}

// Tile sizes and work items for a configuration; uploads the tables.
int32_t batch_configure(BatchState& b, const pcls_batch_config& cfg_in, hipStream_t stream) {
  DeviceLimits lim;
  int32_t st = device_limits(lim);
  if (st != PCLS_OK) return st;
  pcls_batch_config cfg = cfg_in;
  if (cfg.block_threads == 0) cfg.block_threads = 1024;
  if (cfg.block_threads != 256 && cfg.block_threads != 512 && cfg.block_threads != 1024)
    return set_error(PCLS_E_INVALID, "block_threads %d must be 256, 512 or 1024", cfg.block_threads);
  // the persistent kernel keeps one claimed-item word after the tiles
  const int lds_cap = lim.lds_max - 256;
  if (cfg.lds_budget <= 0 || cfg.lds_budget > lds_cap) cfg.lds_budget = lds_cap;
  if (cfg.accumulator_bits != 0 && cfg.accumulator_bits != 32 && cfg.accumulator_bits != 64)
    return set_error(PCLS_E_INVALID, "accumulator_bits must be 0, 32 or 64");
  const size_t budget = (size_t)cfg.lds_budget;
  // accumulator (one width per launch): 64-bit if an instance asks for it or
  // needs it by the automatic rule and every instance fits with it, else 32-bit
  bool acc64 = cfg.accumulator_bits == 64;
  if (cfg.accumulator_bits == 0) {
    bool fits64 = true, asked64 = false, needs64 = false;
    for (const pcls_problem* p : b.probs) {
      if (tile_lds_bytes(state_rows(p), 1, 8) > budget) fits64 = false;
      if (p->acc_bits == 64) asked64 = true;
      if (p->acc_bits == 0 && p->s_g32 < kAcc32MinScale) needs64 = true;
    }
    acc64 = asked64 || (needs64 && fits64);  // an instance that asked and does not fit is rejected below
  }
  const int ab = acc64 ? 8 : 4;
  b.maxb = 0;
  b.items.clear();
  b.inst.resize(b.probs.size());
  size_t lds = 0;
  struct Cost {
    double cost;
    BatchItem it;
  };
  std::vector<Cost> work;
  for (size_t i = 0; i < b.probs.size(); ++i) {
    const pcls_problem* p = b.probs[i];
    if (tile_lds_bytes(state_rows(p), 1, ab) > budget)
      return set_error(PCLS_E_UNSUPPORTED, "instance %zu (%d variables) does not fit the LDS budget of %zu bytes", i,
                       p->n, budget);
    if (!acc64 && p->s_g32 < 8)
      return set_error(PCLS_E_UNSUPPORTED, "instance %zu: weights too large for a 32-bit accumulator", i);
    b.maxb = std::max(b.maxb, p->max_bucket);
    const int R_pad = round_up64(b.R[i]);
    const int tmax_group = kWave / std::max(1, p->max_group);
    int T = 1;
    while (T * 2 <= tmax_group && T * 2 <= R_pad && tile_lds_bytes(state_rows(p), T * 2, ab) <= budget) T *= 2;
    int logT = 0;
    while ((1 << logT) < T) ++logT;
    lds = std::max(lds, tile_lds_bytes(state_rows(p), T, ab));
    for (int r0 = 0; r0 < b.R[i]; r0 += T)
      work.push_back({(double)p->L * T + (double)p->n * T, BatchItem{(int)i, r0, logT, 0}});
    BatchInst& I = b.inst[i];
    I.P = p->dev;
    I.X = b.x[i];
    I.trace = b.trace[i];
    I.R = b.R[i];
    I.ldx = R_pad;
    const int sg = acc64 ? p->s_g64 : p->s_g32;
    I.gsc = std::ldexp(1.0f, sg);
    I.ginv = std::ldexp(1.0f, -sg);
    I.fsc = std::ldexp(1.0f, p->s_f);
    I.finv = std::ldexp(1.0f, -p->s_f);
  }
  std::stable_sort(work.begin(), work.end(), [](const Cost& a, const Cost& c) { return a.cost > c.cost; });
  for (const Cost& w : work) b.items.push_back(w.it);
  b.n_items = (int)b.items.size();
  b.acc64 = acc64;
  b.lds = (lds + 255) / 256 * 256;
  // persistent workgroups: as many per CU as LDS and 16 resident waves allow
  int per_cu = std::max(1, (int)((size_t)lim.lds_max / (b.lds + 256)));
  per_cu = std::min(per_cu, 16 * kWave / cfg.block_threads);
  if (cfg.wgs_per_cu > 0) per_cu = std::min(per_cu, cfg.wgs_per_cu);
  b.grid = std::max(1, std::min(b.n_items, per_cu * std::max(1, lim.n_cu)));
  cfg.wgs_per_cu = per_cu;
  cfg.accumulator_bits = acc64 ? 64 : 32;
  b.cfg = cfg;
  uint8_t* base = (uint8_t*)b.d_ws;
  PCLS_HIP(hipMemcpyAsync(base + b.off_inst, b.inst.data(), sizeof(BatchInst) * b.inst.size(),
                          hipMemcpyHostToDevice, stream),
           "hipMemcpyAsync(batch instances)");
  PCLS_HIP(hipMemcpyAsync(base + b.off_items, b.items.data(), sizeof(BatchItem) * b.items.size(),
                          hipMemcpyHostToDevice, stream),
           "hipMemcpyAsync(batch items)");
  // the host tables must outlive the asynchronous copies
  PCLS_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
  if (b.exec) {
    (void)hipGraphExecDestroy(b.exec);
    b.exec = nullptr;
  }
  if (b.graph) {
    (void)hipGraphDestroy(b.graph);
    b.graph = nullptr;
  }
  return PCLS_OK;
}

int32_t batch_launch(BatchState& b, float lr, int n_steps, hipStream_t stream) {
  uint8_t* base = (uint8_t*)b.d_ws;
  const BatchInst* insts = (const BatchInst*)(base + b.off_inst);
  const BatchItem* items = (const BatchItem*)(base + b.off_items);
  unsigned int* counter = (unsigned int*)(base + b.off_counter);
  // reset the work counter with a kernel (graph-capturable, no memset node)
  hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, stream, counter, 0u, 1);
  PCLS_HIP(hipGetLastError(), "fill launch");
  const dim3 grid(b.grid), block(b.cfg.block_threads);
  if (b.acc64) {
    auto k = b.maxb <= kMaxbShort ? batch_kernel<kMaxbShort, unsigned long long>
                         : (b.maxb <= kMaxbMid ? batch_kernel<kMaxbMid, unsigned long long> : batch_kernel<kMaxbAll, unsigned long long>);
    hipLaunchKernelGGL(k, grid, block, b.lds + 256, stream, insts, items, b.n_items, counter, lr, n_steps,
                       (int)b.lds);
  } else {
    auto k = b.maxb <= kMaxbShort ? batch_kernel<kMaxbShort, unsigned int>
                         : (b.maxb <= kMaxbMid ? batch_kernel<kMaxbMid, unsigned int> : batch_kernel<kMaxbAll, unsigned int>);
    hipLaunchKernelGGL(k, grid, block, b.lds + 256, stream, insts, items, b.n_items, counter, lr, n_steps,
                       (int)b.lds);
  }
  PCLS_HIP(hipGetLastError(), "batch_kernel launch");
  return PCLS_OK;
}

std::mutex g_batch_attr_mu;
bool g_batch_attr_set[64] = {false};

int32_t batch_attrs() {
  int dev = 0;
  PCLS_HIP(hipGetDevice(&dev), "hipGetDevice");
  DeviceLimits lim;
  int32_t st = device_limits(lim);
  if (st != PCLS_OK) return st;
  std::lock_guard<std::mutex> lk(g_batch_attr_mu);
  if (dev >= 0 && dev < 64 && !g_batch_attr_set[dev]) {
    const void* fs[] = {(const void*)batch_kernel<kMaxbShort, unsigned long long>, (const void*)batch_kernel<kMaxbMid, unsigned long long>,
                        (const void*)batch_kernel<kMaxbAll, unsigned long long>, (const void*)batch_kernel<kMaxbShort, unsigned int>,
                        (const void*)batch_kernel<kMaxbMid, unsigned int>, (const void*)batch_kernel<kMaxbAll, unsigned int>};
    for (const void* f : fs) {
      PCLS_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim.lds_max),
               "hipFuncSetAttribute");
      PCLS_HIP(check_no_static_lds(f), "batch kernel attributes");
    }
    g_batch_attr_set[dev] = true;
  }
  return PCLS_OK;
}

// Launches of the per-constraint gradient statistic: zero the accumulator
// (a fill kernel, not a memset node, so the launches can be captured), one
// workgroup per restart, then the conversion to float in the caller's order.
int32_t grad_stats_launch(const pcls_problem* p, int32_t R, const float* d_x, unsigned long long* d_acc,
                          float* d_out, hipStream_t s) {
  DeviceLimits lim;
  int32_t st = device_limits(lim);
  if (st != PCLS_OK) return st;
  const size_t lds = (size_t)((state_rows(p) + 1) & ~1) * 4 + 4 * kMaxSegments;
  if (lds > (size_t)lim.lds_max)
    return set_error(PCLS_E_UNSUPPORTED, "state of %d variables does not fit in LDS", p->n);
  // every term is at most 1, so a constraint's sum over R restarts is at most R k
  const int bits = (int)std::ceil(std::log2((double)R * (double)std::max(1, p->max_k) + 1.0));
  const int sc = std::min(40, 60 - bits);
  hipLaunchKernelGGL(fill_u32_kernel, dim3((2 * p->m + 255) / 256), dim3(256), 0, s, (unsigned int*)d_acc, 0u,
                     2 * p->m);
  PCLS_HIP(hipGetLastError(), "fill launch");
  StatsOut so{d_acc, std::ldexp(1.0f, sc)};
  const int block = p->n > 4096 ? 1024 : 256;
  auto kern = p->max_bucket <= kMaxbShort ? stats_kernel<kMaxbShort> : (p->max_bucket <= kMaxbMid ? stats_kernel<kMaxbMid> : stats_kernel<kMaxbAll>);
  hipLaunchKernelGGL(kern, dim3(R), dim3(block), lds, s, p->dev, d_x, round_up64(R), so);
  PCLS_HIP(hipGetLastError(), "stats_kernel launch");
  hipLaunchKernelGGL(stats_finish_kernel, dim3((p->m + 255) / 256), dim3(256), 0, s, d_acc, p->dev.perm, p->m,
                     std::ldexp(1.0, -sc), d_out);
  PCLS_HIP(hipGetLastError(), "stats_finish launch");
  clear_error();
  return PCLS_OK;
}

// Static scratch of the allocation-free statistic entry point: one 64-bit
// accumulator per constraint, at most kStatsScratchWords (2 MiB), held by each
// device the library runs on until the process ends.  In host code the array's
// name is not a device address: its address on the current device comes from
// hipGetSymbolAddress, looked up once per device and kept.  Every call on a
// device shares that device's array (it is zeroed at the start of each call),
// so calls that overlap on one device race.
constexpr int kStatsScratchWords = 1 << 18;
__device__ __align__(256) unsigned long long scratch[kStatsScratchWords];

std::mutex g_scratch_mu;
unsigned long long* g_scratch_ptr[64] = {};

int32_t stats_scratch(unsigned long long** out) {
  int dev = 0;
  PCLS_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) return set_error(PCLS_E_HIP, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    PCLS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = reinterpret_cast<unsigned long long*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return PCLS_OK;
}

}  // namespace

struct pcls_batch {
  BatchState s;
};

// ======================================================================= C ABI

extern "C" {

int32_t pcls_plan(int32_t n_vars, int32_t n_cons, const int32_t* row_ptr, const int32_t* lit, const int8_t* type,
                  const int32_t* param, const float* weight, pcls_problem** out, size_t* workspace_bytes) {
  return build_plan(n_vars, n_cons, row_ptr, lit, type, param, weight, nullptr, out, workspace_bytes);
}

int32_t pcls_plan_ex(int32_t n_vars, int32_t n_cons, const int32_t* row_ptr, const int32_t* lit,
                     const int8_t* type, const int32_t* param, const float* weight,
                     const pcls_plan_options* options, pcls_problem** out, size_t* workspace_bytes) {
  return build_plan(n_vars, n_cons, row_ptr, lit, type, param, weight, options, out, workspace_bytes);
}

int32_t pcls_problem_info(const pcls_problem* p, pcls_info* info) {
  if (!p || !info) return set_error(PCLS_E_INVALID, "NULL argument");
  std::memset(info, 0, sizeof *info);
  info->n_vars = p->n;
  info->n_cons = p->m;
  info->n_lits = p->L;
  info->max_len = p->max_k;
  info->n_classes = (int32_t)p->classes.size();
  info->n_segments = (int32_t)p->segments.size();
  info->accumulator_bits = p->acc_bits;
  info->grad_scale_log2_64 = p->s_g64;
  info->grad_scale_log2_32 = p->s_g32;
  info->obj_scale_log2 = p->s_f;
  info->tile_restarts = p->tile_restarts;
  info->block_threads = p->block_threads;
  info->workspace_bytes = p->image.size();
  info->lds_bytes_per_restart = (size_t)state_rows(p) * 2 * sizeof(float);
  for (int32_t c : p->c_cls) ++info->cons_by_kind[p->classes[(size_t)c].kind];
  info->bucket_table = p->bucket_table;
  clear_error();
  return PCLS_OK;
}

int32_t pcls_upload(pcls_problem* p, void* d_ws, size_t bytes, void* stream) {
  if (!p) return set_error(PCLS_E_INVALID, "problem handle is NULL");
  if (!d_ws) return set_error(PCLS_E_WORKSPACE, "workspace pointer is NULL");
  if (bytes < p->image.size())
    return set_error(PCLS_E_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes required", bytes,
                     p->image.size());
  if (((uintptr_t)d_ws & 255u) != 0) return set_error(PCLS_E_WORKSPACE, "workspace must be 256-byte aligned");
  PCLS_HIP(hipMemcpyAsync(d_ws, p->image.data(), p->image.size(), hipMemcpyHostToDevice, (hipStream_t)stream),
           "hipMemcpyAsync(workspace)");
  uint8_t* b = (uint8_t*)d_ws;
  ProblemDev& D = p->dev;
  D.n = p->n;
  D.n_pad = p->n_pad;
  D.m = p->m;
  D.L = (int32_t)p->L;
  D.n_segments = (int32_t)p->segments.size();
  D.n_classes = (int32_t)p->classes.size();
  D.f_const = p->f_const;
  D.segments = (const Segment*)(b + p->off_segments);
  D.classes = (const ClassRec*)(b + p->off_classes);
  D.nodes = (const NodeRec*)(b + p->off_nodes);
  D.sp = (const int8_t*)(b + p->off_sp);
  D.litT = (const int32_t*)(b + p->off_litT);
  D.c_k = (const int32_t*)(b + p->off_ck);
  D.c_cls = (const int32_t*)(b + p->off_ccls);
  D.c_w = (const float*)(b + p->off_cw);
  D.row_ptr = (const int32_t*)(b + p->off_rowptr);
  D.lit = (const int32_t*)(b + p->off_lit);
  D.unit_weights = p->unit_weights;
  D.max_k = p->max_k;
  D.occ = (const int32_t*)(b + p->off_occ);
  D.perm = (const int32_t*)(b + p->off_perm);
  p->d_ws = d_ws;
  p->ws_bytes = bytes;
  clear_error();
  return PCLS_OK;
}

int32_t pcls_init_restarts(const pcls_problem* p, int32_t R, uint64_t seed, float* d_x, void* stream) {
  int32_t st = check_bound(p);
  if (st != PCLS_OK) return st;
  if (R < 0) return set_error(PCLS_E_INVALID, "R must be >= 0");
  if (R == 0) return PCLS_OK;
  if (!d_x) return set_error(PCLS_E_INVALID, "d_x is NULL");
  const int R_pad = round_up64(R);
  hipLaunchKernelGGL(init_kernel, dim3(R_pad / 64, p->n), dim3(64), 0, (hipStream_t)stream, d_x, p->n, R, R_pad,
                     (uint32_t)seed, (uint32_t)(seed >> 32), (const uint8_t*)nullptr);
  PCLS_HIP(hipGetLastError(), "init_kernel launch");
  clear_error();
  return PCLS_OK;
}

int32_t pcls_init_restarts_masked(const pcls_problem* p, int32_t R, uint64_t seed, const uint8_t* d_mask, float* d_x,
                                  void* stream) {
  int32_t st = check_bound(p);
  if (st != PCLS_OK) return st;
  if (R < 0) return set_error(PCLS_E_INVALID, "R must be >= 0");
  if (R == 0) return PCLS_OK;
  if (!d_x) return set_error(PCLS_E_INVALID, "d_x is NULL");
  if (!d_mask) return set_error(PCLS_E_INVALID, "d_mask is NULL");
  const int R_pad = round_up64(R);
  hipLaunchKernelGGL(init_kernel, dim3(R_pad / 64, p->n), dim3(64), 0, (hipStream_t)stream, d_x, p->n, R, R_pad,
                     (uint32_t)seed, (uint32_t)(seed >> 32), d_mask);
  PCLS_HIP(hipGetLastError(), "init_kernel launch");
  clear_error();
  return PCLS_OK;
}

int32_t pcls_evaluate(const pcls_problem* p, int32_t R, const float* d_x, float* d_obj, float* d_grad,
                      void* stream) {
  int32_t st = check_bound(p);
  if (st != PCLS_OK) return st;
  if (R < 0) return set_error(PCLS_E_INVALID, "R must be >= 0");
  if (R == 0) return PCLS_OK;
  if (!d_x || !d_obj) return set_error(PCLS_E_INVALID, "d_x and d_obj must not be NULL");
  st = launch_tile(p, R, const_cast<float*>(d_x), 0.f, 1, nullptr, d_obj, d_grad, (hipStream_t)stream);
  if (st == PCLS_OK) clear_error();
  return st;
}

int32_t pcls_step(const pcls_problem* p, int32_t R, float* d_x, float lr, int32_t n_steps, float* d_obj_trace,
                  void* stream) {
  int32_t st = check_bound(p);
  if (st != PCLS_OK) return st;
  if (R < 0 || n_steps < 0) return set_error(PCLS_E_INVALID, "R and n_steps must be >= 0");
  if (!(lr == lr)) return set_error(PCLS_E_INVALID, "lr is NaN");
  if (R == 0 || n_steps == 0) return PCLS_OK;
  if (!d_x) return set_error(PCLS_E_INVALID, "d_x is NULL");
  st = launch_tile(p, R, d_x, lr, n_steps, d_obj_trace, nullptr, nullptr, (hipStream_t)stream);
  if (st == PCLS_OK) clear_error();
  return st;
}

int32_t pcls_step_ex(const pcls_problem* p, int32_t R, float* d_x, float lr, int32_t n_steps, float* d_obj_trace,
                     const pcls_step_options* opt, void* stream) {
  int32_t st = check_bound(p);
  if (st != PCLS_OK) return st;
  if (R < 0 || n_steps < 0) return set_error(PCLS_E_INVALID, "R and n_steps must be >= 0");
  if (!(lr == lr)) return set_error(PCLS_E_INVALID, "lr is NaN");
  if (opt && !(opt->tol >= 0.f)) return set_error(PCLS_E_INVALID, "tol must be >= 0");
  if (R == 0 || n_steps == 0) return PCLS_OK;
  if (!d_x) return set_error(PCLS_E_INVALID, "d_x is NULL");
  st = launch_tile(p, R, d_x, lr, n_steps, d_obj_trace, nullptr, nullptr, (hipStream_t)stream, opt);
  if (st == PCLS_OK) clear_error();
  return st;
}

int32_t pcls_extract(const pcls_problem* p, int32_t R, const float* d_x, int8_t* d_assign, int32_t* d_unsat,
                     int32_t* d_best, void* stream) {
  int32_t st = check_bound(p);
  if (st != PCLS_OK) return st;
  if (R < 0) return set_error(PCLS_E_INVALID, "R must be >= 0");
  if (R == 0) return PCLS_OK;
  if (!d_x || !d_unsat) return set_error(PCLS_E_INVALID, "d_x and d_unsat must not be NULL");
  hipStream_t s = (hipStream_t)stream;
  const int R_pad = round_up64(R);
  hipLaunchKernelGGL(fill_i32_kernel, dim3((R + 255) / 256), dim3(256), 0, s, d_unsat, 0, R);
  PCLS_HIP(hipGetLastError(), "fill launch");
  if (p->m > 0) {
    // threads over restarts (coalesced reads of X), blocks over chunks of
    // constraints; each thread walks its chunk serially, so the chunk is sized
    // for about 1024 waves in total (at least 8 and at most 256 constraints),
    // and a block is no wider than the padded restart count
    const int threads = std::min(256, R_pad);
    const int rblocks = (R + threads - 1) / threads;
    const long long waves_r = (long long)rblocks * (threads / 64);
    const int chunk = (int)std::min<long long>(256, std::max<long long>(8, (long long)p->m * waves_r / 1024));
    hipLaunchKernelGGL(extract_count_kernel, dim3(rblocks, (p->m + chunk - 1) / chunk), dim3(threads), 0, s,
                       p->dev, d_x, R, R_pad, d_unsat, chunk);
    PCLS_HIP(hipGetLastError(), "extract_count launch");
  }
  if (d_assign) {
    hipLaunchKernelGGL(extract_assign_kernel, dim3((R + 63) / 64, (p->n + 63) / 64), dim3(256), 0, s, d_x, p->n, R,
                       R_pad, d_assign);
    PCLS_HIP(hipGetLastError(), "extract_assign launch");
  }
  if (d_best) {
    hipLaunchKernelGGL(extract_best_kernel, dim3(1), dim3(1024), 0, s, d_unsat, R, d_best);
    PCLS_HIP(hipGetLastError(), "extract_best launch");
  }
  clear_error();
  return PCLS_OK;
}

int32_t pcls_constraint_grad_stats(const pcls_problem* p, int32_t R, const float* d_x, uint64_t* d_acc_u64,
                                   float* d_out, void* stream) {
  unsigned long long* d_acc = reinterpret_cast<unsigned long long*>(d_acc_u64);
  int32_t st = check_bound(p);
  if (st != PCLS_OK) return st;
  if (R < 1) return set_error(PCLS_E_INVALID, "R must be >= 1");
  if (p->m == 0) return PCLS_OK;
  if (!d_x || !d_acc || !d_out) return set_error(PCLS_E_INVALID, "d_x, d_acc and d_out must not be NULL");
  return grad_stats_launch(p, R, d_x, d_acc, d_out, (hipStream_t)stream);
}

int32_t pcls_constraint_grad_stats_noalloc(const pcls_problem* p, int32_t R, const float* d_x, float* d_out,
                                           void* stream) {
  int32_t st = check_bound(p);
  if (st != PCLS_OK) return st;
  if (R < 1) return set_error(PCLS_E_INVALID, "R must be >= 1");
  if (p->m == 0) return PCLS_OK;
  if (!d_x || !d_out) return set_error(PCLS_E_INVALID, "d_x and d_out must not be NULL");
  if (p->m > kStatsScratchWords)
    return set_error(PCLS_E_UNSUPPORTED, "%d constraints exceed the %d words of the library's static scratch", p->m,
                     kStatsScratchWords);
  unsigned long long* acc = nullptr;
  st = stats_scratch(&acc);
  if (st != PCLS_OK) return st;
  return grad_stats_launch(p, R, d_x, acc, d_out, (hipStream_t)stream);
}

int32_t pcls_launch_info(const pcls_problem* p, int32_t R, int32_t* tile_restarts, int32_t* block_threads,
                         int32_t* accumulator_bits, int32_t* grad_scale_log2, size_t* lds_bytes) {
  if (!p) return set_error(PCLS_E_INVALID, "problem handle is NULL");
  if (R < 1) return set_error(PCLS_E_INVALID, "R must be >= 1");
  Launch L;
  int32_t st = choose_launch(p, R, L);
  if (st != PCLS_OK) return st;
  if (tile_restarts) *tile_restarts = 1 << L.logT;
  if (block_threads) *block_threads = L.block;
  if (accumulator_bits) *accumulator_bits = L.acc64 ? 64 : 32;
  if (grad_scale_log2) *grad_scale_log2 = L.acc64 ? p->s_g64 : p->s_g32;
  if (lds_bytes) *lds_bytes = L.lds;
  clear_error();
  return PCLS_OK;
}

int32_t pcls_set_launch(pcls_problem* p, int32_t tile_restarts, int32_t block_threads) {
  if (!p) return set_error(PCLS_E_INVALID, "problem handle is NULL");
  if (tile_restarts < 0 || tile_restarts > 64 || (tile_restarts & (tile_restarts - 1)))
    return set_error(PCLS_E_INVALID, "tile_restarts %d must be 0 or a power of two <= 64", tile_restarts);
  if (block_threads != 0 && block_threads != 256 && block_threads != 512 && block_threads != 1024)
    return set_error(PCLS_E_INVALID, "block_threads %d must be 0, 256, 512 or 1024", block_threads);
  if (tile_restarts > 0 && tile_restarts * p->max_group > kWave)
    return set_error(PCLS_E_UNSUPPORTED, "tile_restarts %d too large for constraints of %d literals", tile_restarts,
                     p->max_k);
  if (tile_restarts > 0 && tile_lds_bytes(state_rows(p), tile_restarts, p->acc_bits == 64 ? 8 : 4) > (size_t)160 * 1024)
    return set_error(PCLS_E_UNSUPPORTED, "tile of %d restarts x %d variables exceeds LDS", tile_restarts, p->n);
  p->tile_restarts = tile_restarts;
  p->block_threads = block_threads;
  clear_error();
  return PCLS_OK;
}

int32_t pcls_batch_create(const pcls_problem* const* problems, int32_t count, const int32_t* restarts,
                          pcls_batch** out, size_t* workspace_bytes) {
  if (!out || !workspace_bytes || !problems || !restarts || count < 1)
    return set_error(PCLS_E_INVALID, "NULL argument or empty batch");
  *out = nullptr;
  size_t max_items = 0;
  for (int i = 0; i < count; ++i) {
    if (!problems[i]) return set_error(PCLS_E_INVALID, "problem %d is NULL", i);
    if (!problems[i]->d_ws) return set_error(PCLS_E_WORKSPACE, "problem %d has no device workspace", i);
    if (restarts[i] < 1) return set_error(PCLS_E_INVALID, "restarts[%d] must be >= 1", i);
    max_items += (size_t)restarts[i];
  }
  pcls_batch* b = new (std::nothrow) pcls_batch();
  if (!b) return set_error(PCLS_E_INVALID, "out of host memory");
  b->s.probs.assign(problems, problems + count);
  b->s.R.assign(restarts, restarts + count);
  b->s.x.assign(count, nullptr);
  b->s.trace.assign(count, nullptr);
  size_t off = 0;
  auto place = [&](size_t bytes) {
    off = (off + 255) / 256 * 256;
    size_t at = off;
    off += bytes;
    return at;
  };
  b->s.off_inst = place(sizeof(BatchInst) * (size_t)count);
  b->s.off_items = place(sizeof(BatchItem) * max_items);
  b->s.off_counter = place(256);
  b->s.ws_bytes = batch_ws_bytes(count, max_items);
  *out = b;
  *workspace_bytes = b->s.ws_bytes;
  clear_error();
  return PCLS_OK;
}

int32_t pcls_batch_bind(pcls_batch* b, void* d_ws, size_t bytes, float* const* d_x, float* const* d_trace,
                        void* stream) {
  if (!b || !d_x) return set_error(PCLS_E_INVALID, "NULL argument");
  if (!d_ws || bytes < b->s.ws_bytes || ((uintptr_t)d_ws & 255u))
    return set_error(PCLS_E_WORKSPACE, "batch workspace missing, misaligned or smaller than %zu bytes", b->s.ws_bytes);
  for (size_t i = 0; i < b->s.probs.size(); ++i) {
    if (!d_x[i]) return set_error(PCLS_E_INVALID, "state %zu is NULL", i);
    b->s.x[i] = d_x[i];
    b->s.trace[i] = d_trace ? d_trace[i] : nullptr;
  }
  b->s.d_ws = d_ws;
  int32_t st = batch_attrs();
  if (st != PCLS_OK) return st;
  st = batch_configure(b->s, b->s.cfg, (hipStream_t)stream);
  if (st == PCLS_OK) clear_error();
  return st;
}

int32_t pcls_batch_set_config(pcls_batch* b, const pcls_batch_config* cfg, void* stream) {
  if (!b || !cfg) return set_error(PCLS_E_INVALID, "NULL argument");
  if (!b->s.d_ws) return set_error(PCLS_E_WORKSPACE, "batch is not bound (call pcls_batch_bind)");
  int32_t st = batch_configure(b->s, *cfg, (hipStream_t)stream);
  if (st == PCLS_OK) clear_error();
  return st;
}

int32_t pcls_batch_get_config(const pcls_batch* b, pcls_batch_config* cfg, int32_t* n_items, int32_t* grid) {
  if (!b) return set_error(PCLS_E_INVALID, "NULL argument");
  if (cfg) *cfg = b->s.cfg;
  if (n_items) *n_items = b->s.n_items;
  if (grid) *grid = b->s.grid;
  clear_error();
  return PCLS_OK;
}

int32_t pcls_batch_step(pcls_batch* b, float lr, int32_t n_steps, void* stream) {
  if (!b) return set_error(PCLS_E_INVALID, "NULL argument");
  if (!b->s.d_ws) return set_error(PCLS_E_WORKSPACE, "batch is not bound (call pcls_batch_bind)");
  if (n_steps < 0 || !(lr == lr)) return set_error(PCLS_E_INVALID, "bad n_steps or lr");
  if (n_steps == 0) return PCLS_OK;
  int32_t st = batch_launch(b->s, lr, n_steps, (hipStream_t)stream);
  if (st == PCLS_OK) clear_error();
  return st;
}

int32_t pcls_batch_capture(pcls_batch* b, float lr, int32_t n_steps, void* stream) {
  if (!b) return set_error(PCLS_E_INVALID, "NULL argument");
  if (!b->s.d_ws) return set_error(PCLS_E_WORKSPACE, "batch is not bound (call pcls_batch_bind)");
  if (n_steps < 1 || !(lr == lr)) return set_error(PCLS_E_INVALID, "bad n_steps or lr");
  BatchState& s = b->s;
  if (!s.cap_stream) PCLS_HIP(hipStreamCreateWithFlags(&s.cap_stream, hipStreamNonBlocking), "hipStreamCreate");
  // order the capture after work already queued on the caller's stream
  PCLS_HIP(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
  if (s.exec) {
    (void)hipGraphExecDestroy(s.exec);
    s.exec = nullptr;
  }
  if (s.graph) {
    (void)hipGraphDestroy(s.graph);
    s.graph = nullptr;
  }
  PCLS_HIP(hipStreamBeginCapture(s.cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  int32_t st = batch_launch(s, lr, n_steps, s.cap_stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s.cap_stream, &g);
  if (st != PCLS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  s.graph = g;
  PCLS_HIP(hipGraphInstantiate(&s.exec, s.graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  clear_error();
  return PCLS_OK;
}

int32_t pcls_batch_replay(pcls_batch* b, void* stream) {
  if (!b) return set_error(PCLS_E_INVALID, "NULL argument");
  if (!b->s.exec) return set_error(PCLS_E_INVALID, "no captured graph (call pcls_batch_capture)");
  PCLS_HIP(hipGraphLaunch(b->s.exec, (hipStream_t)stream), "hipGraphLaunch");
  clear_error();
  return PCLS_OK;
}

int32_t pcls_batch_autotune(pcls_batch* b, float lr, int32_t probe_steps, void* stream, pcls_batch_config* best,
                            float* best_ms) {
  if (!b || probe_steps < 1) return set_error(PCLS_E_INVALID, "NULL batch or probe_steps < 1");
  if (!b->s.d_ws) return set_error(PCLS_E_WORKSPACE, "batch is not bound (call pcls_batch_bind)");
  DeviceLimits lim;
  int32_t st = device_limits(lim);
  if (st != PCLS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  PCLS_HIP(hipEventCreate(&e0), "hipEventCreate");
  PCLS_HIP(hipEventCreate(&e1), "hipEventCreate");
  const int blocks[] = {256, 512, 1024};
  const int budgets[] = {lim.lds_max, lim.lds_max / 2, lim.lds_max / 3, lim.lds_max / 4};
  pcls_batch_config win{};
  float win_ms = 0.f;
  bool have = false;
  for (int bt : blocks) {
    for (int bud : budgets) {
      pcls_batch_config c{};
      c.block_threads = bt;
      c.lds_budget = bud;
      c.accumulator_bits = b->s.cfg.accumulator_bits == 32 ? 32 : 0;
      if (batch_configure(b->s, c, s) != PCLS_OK) continue;  // infeasible budget
      if (batch_launch(b->s, lr, 1, s) != PCLS_OK) continue;  // warm-up
      (void)hipEventRecord(e0, s);
      st = batch_launch(b->s, lr, probe_steps, s);
      (void)hipEventRecord(e1, s);
      if (st != PCLS_OK) continue;
      if (hipEventSynchronize(e1) != hipSuccess) continue;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (!have || ms < win_ms) {
        win = b->s.cfg;
        win_ms = ms;
        have = true;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!have) return set_error(PCLS_E_UNSUPPORTED, "no feasible batch configuration");
  st = batch_configure(b->s, win, s);
  if (st != PCLS_OK) return st;
  if (best) *best = b->s.cfg;
  if (best_ms) *best_ms = win_ms;
  clear_error();
  return PCLS_OK;
}

int32_t pcls_batch_destroy(pcls_batch* b) {
  delete b;
  return PCLS_OK;
}

int32_t pcls_destroy(pcls_problem* p) {
  delete p;
  return PCLS_OK;
}

const char* pcls_last_error(void) { return pcls::last_error(); }

}  // extern "C"
