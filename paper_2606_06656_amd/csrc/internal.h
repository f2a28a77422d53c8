// Internal layout shared by the host planner and the gfx950 kernels.
//
// A planned problem is one contiguous device image (caller-owned workspace).
// Constraints are reordered into segments; each segment holds constraints of
// one evaluation kind and one length bucket, so a wavefront runs one code path.
#pragma once
#include <cstddef>
#include <cstdint>

namespace pcls {

// Evaluation kinds.  Every kind evaluates FE = sum_t sp_t Pr[T = t] (T = number
// of true literals under independent literals of mean y) through products of
// per-literal factors (alpha + beta * y) at a set of nodes:
//   PROD1 - one real node (sp constant except at t = 0, t = k, or alternating):
//           FE = c0 + c1 * prod_i (a + b y_i)
//   PROD2 - two real nodes (sp constant on 1..k-1):
//           FE = c0 + c1 * prod_i (1+y_i)/2 + c2 * prod_i (1-y_i)/2
//   DFT   - the K = k+1 complex roots of unity: FE = sum_m chat_m prod_i(alpha_m + beta_m y_i)
//   PMF   - sp constant outside a window of w counts at one end (thresholds,
//           at-most-one, exactly-kappa near an end), w <= 4 for k <= 8 (one lane
//           per pair) and w <= KMAX/2 of the length bucket for 8 < k <= 48 (lane
//           groups): with C the number of true literals (or of false ones),
//           FE = c0 + sum_{c < w} d_c Pr[C = c], from a truncated Poisson-binomial
//           recursion and its adjoint (no products of complex factors)
//   CONST - sp constant: FE = c0, no literal work
enum Kind : int32_t { KIND_PROD1 = 0, KIND_PROD2 = 1, KIND_DFT = 2, KIND_PMF = 3, KIND_CONST = 4 };
constexpr int kNumKinds = 5;
constexpr int kPmfWindow = 4;  // counts kept by the PMF kind, one lane per pair (k <= 8)
constexpr int kPmfMaxK = 8;    // longest constraint of the one-lane PMF kind
constexpr int kPmfGroupMaxK = 48;  // longest constraint of the lane-group PMF kind (window <= bucket / 2)

// Length buckets of the segment kernels: literals per constraint padded to KMAX,
// processed by groups of G lanes holding J = KMAX / G literals each.
constexpr int kNumBuckets = 18;
constexpr int kBucketKmax[kNumBuckets] = {1, 2, 3, 4, 5, 6, 7, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256};
// Kernel variants, by the longest bucket they are compiled for.
constexpr int kMaxbShort = 7;                // k <= 8
constexpr int kMaxbMid = 11;                 // k <= 32
constexpr int kMaxbAll = kNumBuckets - 1;    // k <= 256
constexpr int kMaxK = 256;
constexpr int kMaxSegments = 4 * kNumBuckets;  // (kind, bucket) pairs of the non-constant kinds
// Pad rows: problems with constraints longer than 8 literals get kPadRows extra
// rows in the on-chip state, held at x = +1 and never stepped.  A slot past a
// constraint's end (length buckets above 8) codes one of these rows, with the
// literal sign chosen so that the slot's factor is exactly 1 (its gradient
// term lands in the pad row, whose accumulator is never read).  Slot i of
// constraint q of a segment starts on pad row (q + i) mod kPadRows, so pads
// spread over banks; the planner's bank balance may then move them between
// the constraint's slots.
constexpr int kPadRows = 64;

// Lanes per (constraint, restart) pair: one lane holds up to 16 literals of a
// product kind or 8 of the DFT and PMF kinds (register budget at 4 waves per SIMD);
// longer constraints spread over G lanes (a power of two) of at most 8 literals
// each (6 for the buckets 12, 24, ..., 192).
constexpr int lane_groups(int kmax) {
  int g = 1;
  while (kmax > 8 * g) g *= 2;
  return g;
}
constexpr int group_size(int kind, int kmax) {
  return (kmax <= 8 || (kind != KIND_DFT && kind != KIND_PMF && kmax <= 16)) ? 1 : lane_groups(kmax);
}

// Bucket tables: which of the compiled lengths a plan uses.  Table 0 uses all of
// them; table 1 only the exact ones up to 8 and the powers of two above (fewer
// segments, more padded slots).  The autotuners choose between them.
constexpr int kNumBucketTables = 2;
inline bool bucket_in_table(int b, int table) {
  const int k = kBucketKmax[b];
  return table == 0 || k <= 8 || (k & (k - 1)) == 0;
}
inline int bucket_of(int k, int table = 0) {
  for (int b = 0; b < kNumBuckets; ++b)
    if (k <= kBucketKmax[b] && bucket_in_table(b, table)) return b;
  return -1;
}

struct Segment {
  int32_t kind;       // Kind
  int32_t bucket;     // index into kBucketKmax
  int32_t c_begin;    // first constraint (planned order)
  int32_t c_count;    // constraints in the segment
  int32_t lit_base;   // offset of the segment's transposed literal block
  int32_t k_fixed;    // > 0 when every constraint has this length
  int32_t cls_fixed;  // >= 0 when every constraint has this class
  int32_t m_max;      // DFT: largest number of complex nodes; PMF: widest window over the segment
};

// Per constraint class (type, k, param).
struct ClassRec {
  int32_t kind;
  int32_t k;
  int32_t n_nodes;   // DFT: complex nodes m = 1..n_nodes
  int32_t node_off;  // DFT: offset into the node table (entries)
  int32_t nyquist;   // DFT: 1 when K = k + 1 is even (real node at omega = -1); PMF: window w
  int32_t sp_off;    // offset of sp[0..k] (int8) in the spectrum table
  float a, b;        // PROD1 node factor a + b y
  float c1, c2;      // PROD1 / PROD2 product weights; DFT: c1 = chat_{K/2} (Nyquist weight)
  float c0;          // constant term (folded into the per-problem constant on device)
  float pad;
};

// DFT node m of a class: factor alpha + beta y, weight 2*chat_m for the value
// and 2*chat_m*beta_m for the gradient (the 2 covers the conjugate node K - m).
// A PMF class of k <= 8 literals has one record: {d_0, d_1, d_2, d_3, h, 0, 0, 0},
// where the counted event of literal i has probability 1/2 - h y_i (h = 1/2:
// true, -1/2: false); a longer one has five records read as 40 floats:
// d_0..d_31 (zero past its window), h, a threshold flag (d constant on the
// window), then padding.
struct NodeRec {
  float ar, ai, br, bi;
  float wr, wi, gr, gi;
};

// Device view of a planned problem (passed by value to kernels).
struct ProblemDev {
  int32_t n, m, L;
  int32_t n_pad;                 // pad rows after the n variables (0 or kPadRows)
  int32_t n_segments;
  int32_t n_classes;
  float f_const;                 // sum_c w_c c0_c
  const Segment* segments;
  const ClassRec* classes;
  const NodeRec* nodes;
  const int8_t* sp;              // spectra
  const int32_t* litT;           // per segment: [KMAX][c_count] literal codes: variable in bits 0..30,
                                 // bit 31 set for a negated literal; a slot past the constraint's
                                 // end codes a pad row (variable >= n)
  const int32_t* c_k;            // per constraint length (planned order)
  const int32_t* c_cls;          // per constraint class
  const float* c_w;              // per constraint weight
  const int32_t* row_ptr;        // planned-order CSR (extract / streaming engine)
  const int32_t* lit;            // planned-order literal codes
  int32_t unit_weights;          // all weights 1.0
  int32_t max_k;
  const int32_t* occ;            // per variable: occurrences in non-constant constraints
  const int32_t* perm;           // planned index -> caller's constraint index
};

}  // namespace pcls
