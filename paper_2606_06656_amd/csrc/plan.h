// Host-side plan of a formula: validated constraints, classes, segments and the
// device image that pcls_upload copies into the caller's workspace.
#pragma once
#include <cstdarg>
#include <string>
#include <vector>

#include "../../include/pcls.h"
#include "internal.h"

struct pcls_problem {
  int32_t n = 0, m = 0;
  int64_t L = 0;
  int32_t max_k = 0;
  int32_t force_generic = 0;

  std::vector<pcls::Segment> segments;
  std::vector<pcls::ClassRec> classes;
  std::vector<pcls::NodeRec> nodes;
  std::vector<int8_t> sp;
  std::vector<int32_t> litT;
  std::vector<int32_t> c_k, c_cls;
  std::vector<float> c_w;
  std::vector<int32_t> row_ptr, lit;   // planned order
  std::vector<int32_t> perm;           // planned index -> original constraint index
  std::vector<int32_t> occ;            // per variable: occurrences in non-constant constraints
  int32_t max_group = 1;               // largest lane group G over the segments
  int32_t max_bucket = -1;             // largest length bucket over the segments
  int32_t n_pad = 0;                   // pad rows of the on-chip state (kPadRows when max_bucket > 8)
  int32_t bucket_table = 0;            // length-bucket table (see bucket_in_table)
  float f_const = 0.f;
  int32_t unit_weights = 1;

  // fixed-point accumulation: |dFE/dy| <= 1 and |FE| <= 1, so a variable's
  // gradient is bounded by the sum of |w| over its occurrences and the
  // objective by the sum of |w| over constraints
  double maxsum_g = 0.0, max_w = 0.0, maxsum_f = 0.0;
  int32_t acc_bits = 0;   // requested accumulator width (0 = automatic)
  int32_t s_g64 = 0, s_g32 = 0, s_f = 0;

  // device image
  std::vector<uint8_t> image;
  size_t off_segments = 0, off_classes = 0, off_nodes = 0, off_sp = 0, off_litT = 0, off_ck = 0,
         off_ccls = 0, off_cw = 0, off_rowptr = 0, off_lit = 0, off_occ = 0, off_perm = 0;
  void* d_ws = nullptr;
  size_t ws_bytes = 0;
  pcls::ProblemDev dev{};

  // launch settings of the resident engine (0 = automatic)
  int32_t tile_restarts = 0;
  int32_t block_threads = 0;
};

namespace pcls {
int32_t set_error(int32_t code, const char* fmt, ...);
void clear_error();
int32_t build_plan(int32_t n_vars, int32_t n_cons, const int32_t* row_ptr, const int32_t* lit,
                   const int8_t* type, const int32_t* param, const float* weight,
                   const pcls_plan_options* options, pcls_problem** out, size_t* workspace_bytes);
}  // namespace pcls
