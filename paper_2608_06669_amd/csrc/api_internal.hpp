// Handle state behind the C boundary (shared by api.hip and server.hip).
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "../../include/pnkcc.h"
#include "ccsd.hpp"
#include "gauge.hpp"
#include "solvers.hpp"

namespace pnk {

struct ProblemKey {
  int o = 0, v = 0, naux = 0;
  const void *f_oo = nullptr, *f_ov = nullptr, *f_vv = nullptr, *L = nullptr;
  uint64_t hash[4] = {0, 0, 0, 0};
  bool operator==(const ProblemKey& k) const {
    return o == k.o && v == k.v && naux == k.naux && f_oo == k.f_oo && f_ov == k.f_ov && f_vv == k.f_vv &&
           L == k.L && hash[0] == k.hash[0] && hash[1] == k.hash[1] && hash[2] == k.hash[2] && hash[3] == k.hash[3];
  }
};

struct Handle {
  int device = 0;
  size_t limit = 0;
  hipStream_t alloc_stream = nullptr;  // serving workers allocate stream-ordered
  bool stream_ordered = false;
  std::unique_ptr<Engine> eng;
  std::unique_ptr<Solver> sol;
  int sol_m = 0, sol_r = 0, sol_d = 0;
  int64_t sol_cap = 0;   // outer vector length of the solver, if a gauge's
  double* xa = nullptr;  // packed vectors
  double* xb = nullptr;
  uint64_t* hash_buf = nullptr;
  bool prepared = false;
  ProblemKey cached_key;
  std::vector<double> history;
  std::string err;
  std::unique_ptr<Timers> timers;  // set when diagnostics timing is on
  Gauge gauge;                      // buffers of the non-orthogonal gauge entry points
  double* gauge_mem = nullptr;
  ~Handle();
  // Size the gauge buffers for the engine's (o, v) and g's (m_occ, m_vir),
  // grow the solver's outer vectors to the gauge's length, and fill the
  // gauge's matrices from g and the prepared problem's Fock blocks (after
  // ensure()).
  Gauge* ensure_gauge(const cc_gauge* g, hipStream_t s);
  void* dev_alloc(size_t bytes);
  void dev_free(void* p);
  // Size the engine/solver for p and (re)prepare its integrals if the
  // problem's pointers, sizes or content changed.
  void ensure(const cc_problem* p, int lowp, int m_max, int restart, int diis, hipStream_t s);
};

// outer_cap: length of the solver's outer vectors when above the orbital
// one (a redundant gauge's)
size_t workspace_bytes(int o, int v, int naux, int lowp, int m_max, int restart, int diis, int64_t outer_cap = 0);
// Scratch sizes of the batched diagnostic product: split-K partial sums
// (elements, at most kDiagSplitElems) and rounded operand copies (bytes).
constexpr int64_t kDiagSplitElems = int64_t(4) << 20;
int64_t diag_splitk_elems(int64_t nbatch, int M, int N);
int64_t diag_cast_bytes(int64_t nbatch, int M, int N, int K, cc_precision prec);
void check_problem(const cc_problem* p);
void check_pnk_opts(const cc_pnk_opts& o);
PnkOptions to_internal(const cc_pnk_opts& o);
int lowp_for(cc_precision p);

}  // namespace pnk
