// MGRIT solve drivers of libmgrit: the iteration of Sec. 2.2 with the
// multilevel V- and F-cycles of Sec. 4.4, for one plan (mgrit_solve) or for
// several plans on one stream stepped together (mgrit_solve_batch), whose
// relaxation launches are then merged per pass (Batch in plan.h).
//
// Every driver below works on a list of members.  A step records the same
// operation for each member still running, then flushes; a member that
// converges, diverges or fails leaves the lists and the others go on.  With
// one member nothing is recorded: launches go straight to the stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/mgrit.h"
#include "plan.h"
#include "registry.h"

namespace mgr {
namespace {

struct Member {
  Plan* P = nullptr;
  // arguments
  const double* u0 = nullptr;
  const double* uinit = nullptr;
  double tol = 0.0;
  int maxit = 0;
  double* u_out = nullptr;
  int out_kind = MGRIT_OUT_NONE;
  double* hist = nullptr;
  // state
  double* cur = nullptr;
  double* nxt = nullptr;
  const double* corr = nullptr;
  int it = 0;             // coarse corrections applied (outer steps for IR)
  int inner_total = 0;    // IR: inner corrections
  int k = 0;              // IR: inner step
  double res = 0.0, prev = 0.0;
  bool done = false;      // converged / diverged / out of iterations
  bool inner = false;     // IR: inside an inner solve
  int status = MGRIT_ENOTCONV;
  int rc = MGRIT_OK;      // error of a launch or copy (ends the member)
};

typedef std::vector<Member*> List;

bool alive(const Member* M) { return M->rc == MGRIT_OK && !M->done; }

class Group {
 public:
  Group(hipStream_t s, bool record) : stream_(s), record_(record) { batch_.stream = s; }

  void attach(List& all) {
    for (Member* M : all) M->P->batch = record_ ? &batch_ : nullptr;
  }
  void detach(List& all) {
    for (Member* M : all) M->P->batch = nullptr;
  }
  // issue what the step recorded; a launch error ends every member of it
  void flush(const List& l) {
    if (!record_) return;
    const int rc = batch_.flush();
    if (rc)
      for (Member* M : l) fail(M, rc);
  }
  static void fail(Member* M, int rc) {
    if (M->rc == MGRIT_OK) M->rc = rc;
  }
  static void check(Member* M, int rc) {
    if (rc) fail(M, rc);
  }
  // ||r|| of each member from its partial sums (fixed-order reduction), one
  // host synchronisation for all
  void norms(const List& l) {
    for (Member* M : l) {
      Plan* P = M->P;
      hipEvent_t e0 = nullptr;
      if (P->profiling) {
        P->tag = ProfTag();
        P->tag.pass = MGRIT_PASS_NORM;
        P->tag.bytes = P->parts * 8.0;
        P->tag.flops = P->parts;
      }
      P->mark_util(MGRIT_PROF_NORM, e0);
      launch_norm_reduce(P->partial, P->parts, P->scale * P->scale, P->d_norm, stream_);
      P->end_util(MGRIT_PROF_NORM, e0);
      check(M, hipMemcpyAsync(P->h_norm, P->d_norm, sizeof(double), hipMemcpyDeviceToHost,
                              stream_) == hipSuccess ? MGRIT_OK : MGRIT_EHIP);
    }
    const bool ok = hipStreamSynchronize(stream_) == hipSuccess;
    for (Member* M : l) {
      if (!ok) fail(M, MGRIT_EHIP);
      M->res = *M->P->h_norm;
    }
  }
  hipStream_t stream() const { return stream_; }
  const Batch& batch() const { return batch_; }

 private:
  hipStream_t stream_;
  bool record_;
  Batch batch_;
};

List live(const List& l) {
  List o;
  for (Member* M : l)
    if (alive(M)) o.push_back(M);
  return o;
}

// ---- coarse levels ----------------------------------------------------------
// Right-hand side of level l's error system: the C-point residuals of level
// l-1.
const double* rhs_of(const Member* M, int l) { return M->P->lev[l - 1].R; }

// How a cycle on level l starts: from a zero guess, from the guess lev[l].X
// (all points), or from the C-points lev[l].V corrected by lev[l+1].X (what
// an interpolation would leave at the C-points).
enum Start { START_ZERO, START_GUESS, START_CORRECTED };

void cycle(Group& G, const List& l0, int l, Start start, int kind, int prec, bool interpolate);

// Solve level l's error system (zero initial guess) into lev[l].X: on the
// coarsest level by the sequential sweep, else by one V-cycle or by an
// F-cycle followed by a V-cycle.
void coarse_solve(Group& G, const List& l0, int l, int kind, int prec) {
  List seq, rest;
  for (Member* M : live(l0)) (l == (int)M->P->lev.size() - 1 ? seq : rest).push_back(M);
  // spectral solves first (direct launches), then the chunked sweeps
  List sweep;
  for (Member* M : seq) {
    Plan* P = M->P;
    if (!P->spectral) {
      sweep.push_back(M);
      continue;
    }
    Level& L = P->lev.back();
    hipEvent_t e0 = nullptr;
    if (P->profiling) {
      // right-hand side rows in, solution rows out; two real transforms of
      // 2.5 n_x log2 n_x flops per row and a complex multiply-add per mode
      // and step
      P->tag = ProfTag();
      P->tag.level = (int)P->lev.size() - 1;
      P->tag.pass = MGRIT_PASS_SPECTRAL;
      P->tag.bytes = 2.0 * L.n * P->nx * 8.0;
      P->tag.flops = (double)L.n * P->nx * (5.0 * std::log2((double)P->nx) + 8.0);
    }
    P->mark_util(MGRIT_PROF_COARSEST, e0);
    Group::check(M, launch_spectral_solve(rhs_of(M, l), L.X, P->Sspec, L.seq.d_mu,
                                          L.seq.d_tw, P->nx, L.n, G.stream()) == 0
                        ? MGRIT_OK : MGRIT_EHIP);
    P->end_util(MGRIT_PROF_COARSEST, e0);
  }
  seq.swap(sweep);
  if (!seq.empty()) {
    // chunked sequential sweep: one launch per member per round
    std::vector<int> s0(seq.size(), 0);
    for (;;) {
      List round;
      for (size_t i = 0; i < seq.size(); ++i) {
        Member* M = seq[i];
        if (!alive(M) || s0[i] < 0) continue;
        bool last = false;
        Group::check(M, M->P->sequential_chunk(s0[i], rhs_of(M, l), &last));
        const Level& L = M->P->lev.back();
        const int S = L.seq.seq_chunk > 0 ? L.seq.seq_chunk : L.n;
        s0[i] = last ? -1 : s0[i] + S;
        round.push_back(M);
      }
      if (round.empty()) break;
      G.flush(round);
    }
  }
  if (rest.empty()) return;
  if (kind == MGRIT_CYCLE_F) {
    // The V-cycle's relaxation starts from the C-points and recomputes every
    // F-point: of the F-cycle's interpolation only the corrected C-points
    // v + e matter, and the V-cycle forms them as it reads them.
    cycle(G, rest, l, START_ZERO, MGRIT_CYCLE_F, prec, false);
    cycle(G, rest, l, START_CORRECTED, MGRIT_CYCLE_V, prec, true);
  } else {
    cycle(G, rest, l, START_ZERO, MGRIT_CYCLE_V, prec, true);
  }
}

// One V- or F-cycle on level l >= 1 (Sec. 4.4): relax, residual, coarse
// solve, correct + F-relax (the last step left out when `interpolate` is
// false: lev[l].V and lev[l+1].X then hold the relaxed C-points and their
// correction).
//
// With FCF the C-point residual needs no right-hand side rows: the FC pass
// gives v_{j+1} = Psi^m x_j + h_j (h_j the interval's propagated right-hand
// side), so r_{j+1} = Psi^m v_j + h_j - v_{j+1} = Psi^m (v_j - x_j).  The FC
// pass also writes the update d = v - x, and the residual pass propagates d
// alone: m right-hand side rows per interval less to read.  d is held in
// lev[l+1].X, which the coarse solve overwrites only afterwards.
//
// START_CORRECTED reads x = lev[l].V + lev[l+1].X, so the relaxed C-points
// go to lev[l].W and d to lev[l].X (both unused until the interpolation).
void cycle(Group& G, const List& l0, int l, Start start, int kind, int prec, bool interpolate) {
  List a = live(l0);
  const bool corrected = start == START_CORRECTED;
  for (Member* M : a) {
    Plan* P = M->P;
    Level& L = P->lev[l];
    const double* guess = start == START_ZERO ? nullptr : corrected ? L.V : L.X;
    const long long stride = corrected ? 1 : P->m;
    const double* corr = corrected ? P->lev[l + 1].X : nullptr;
    double* v = corrected ? L.W : L.V;
    if (P->relax_kind == MGRIT_RELAX_FCF)
      Group::check(M, P->relax(l, prec, MODE_FC, guess, stride, corr, rhs_of(M, l), RHS_EVERY,
                               v, nullptr, P->m, corrected ? L.X : P->lev[l + 1].X));
    else  // F-relaxation only: v = u
      Group::check(M, P->copy_cpoints(l, prec, guess, stride, corr, v));
  }
  G.flush(a);
  a = live(a);
  for (Member* M : a) {
    Plan* P = M->P;
    Level& L = P->lev[l];
    if (P->relax_kind == MGRIT_RELAX_FCF)
      Group::check(M, P->relax(l, prec, MODE_FC, corrected ? L.X : P->lev[l + 1].X, 1, nullptr,
                               nullptr, RHS_NONE, L.R, nullptr, P->m));
    else
      Group::check(M, P->relax(l, prec, MODE_RES, corrected ? L.W : L.V, 1, nullptr,
                               rhs_of(M, l), RHS_EVERY, L.R, nullptr, P->m));
  }
  G.flush(a);
  coarse_solve(G, a, l + 1, kind, prec);
  if (!interpolate) return;
  a = live(a);
  for (Member* M : a) {
    Plan* P = M->P;
    Level& L = P->lev[l];
    Group::check(M, P->relax(l, prec, MODE_F, corrected ? L.W : L.V, 1, P->lev[l + 1].X,
                             rhs_of(M, l), RHS_EVERY, L.X, nullptr, P->m));
  }
  G.flush(a);
}

// The correction of the fine level by level 2, split by cycle kind.
void correct(Group& G, const List& l0, int prec) {
  List v, f;
  for (Member* M : live(l0)) (M->P->cycle_kind == MGRIT_CYCLE_F ? f : v).push_back(M);
  if (!f.empty()) coarse_solve(G, f, 1, MGRIT_CYCLE_F, prec);
  if (!v.empty()) coarse_solve(G, v, 1, MGRIT_CYCLE_V, prec);
}

// ---- start and end ----------------------------------------------------------
int init_iterate(Plan* P, const double* u0, const double* uinit, double* dst) {
  const int nx = P->nx, nc = P->nt / P->m;
  const size_t row = (size_t)nx * sizeof(double);
  if (uinit) {
    if (hipMemcpyAsync(dst, uinit, row * (nc + 1), hipMemcpyDeviceToDevice, P->stream) !=
        hipSuccess)
      return MGRIT_EHIP;
  } else {
    launch_uniform_init(dst, nc + 1, nx, P->seed, P->stream);
  }
  return hipMemcpyAsync(dst, u0, row, hipMemcpyDeviceToDevice, P->stream) == hipSuccess
             ? MGRIT_OK : MGRIT_EHIP;
}

int finish_output(Plan* P, const double* C, double* u_out, int out_kind) {
  const int nx = P->nx, nc = P->nt / P->m;
  const size_t row = (size_t)nx * sizeof(double);
  switch (out_kind) {
    case MGRIT_OUT_NONE: return MGRIT_OK;
    case MGRIT_OUT_FINAL:
      return hipMemcpyAsync(u_out, C + (size_t)nc * nx, row, hipMemcpyDeviceToDevice,
                            P->stream) == hipSuccess ? MGRIT_OK : MGRIT_EHIP;
    case MGRIT_OUT_CPOINTS:
      return hipMemcpyAsync(u_out, C, row * (nc + 1), hipMemcpyDeviceToDevice, P->stream) ==
                     hipSuccess ? MGRIT_OK : MGRIT_EHIP;
    case MGRIT_OUT_ALL:
      // F-relaxation of the converged C-points on the fine level, in FP64
      return P->relax(0, 0, MODE_F, C, 1, nullptr, nullptr, RHS_NONE, u_out, nullptr, P->m);
    default: return MGRIT_EINVAL;
  }
}

// Record the residual test of member M (hist, stats) and whether it stops.
void judge(Member* M, int idx) {
  Plan* P = M->P;
  if (M->hist) M->hist[idx] = M->res;
  P->stats.final_residual = M->res;
  if (!std::isfinite(M->res)) {
    M->status = MGRIT_EDIVERGED;
    M->done = true;
  } else if (M->res <= M->tol) {
    M->status = MGRIT_OK;
    M->done = true;
  } else if (M->it >= M->maxit) {
    M->status = MGRIT_ENOTCONV;
    M->done = true;
  }
}

// ---- the three solves ---------------------------------------------------------
// FP64 (FCF or F-relaxation), and FP32 relaxation with FCF in correction
// form: with u the current C-points (cur + corr), the FCF-relaxed iterate of
// the FP64 solver is v = FC(u) and its residual r_{j+1} = Phi^m v_j -
// v_{j+1}.  Writing v = u + d (d the C-relaxation update, d^0 = 0) gives
// exactly r_{j+1} = Phi^m d_j, because Phi^m u_j = v_{j+1}: the second fine
// pass acts only on the small update d -- formed in FP64 from v, cur and
// corr as it starts -- and runs in FP32 with errors relative to |d|, while
// the C-point iterate, its FC pass, the coarse correction and the norms
// stay FP64.  Iteration by iteration this is the FP64 solver.
void solve_plain(Group& G, const List& all, bool mixed) {
  for (Member* M : all) {
    Plan* P = M->P;
    Group::check(M, init_iterate(P, M->u0, M->uinit, P->Va));
    M->cur = P->Va;
    M->nxt = P->Vb;
    M->corr = nullptr;
  }
  for (;;) {
    List a = live(all);
    if (a.empty()) break;
    for (Member* M : a) {
      Plan* P = M->P;
      if (mixed || P->relax_kind == MGRIT_RELAX_FCF) {
        Group::check(M, P->relax(0, 0, MODE_FC, M->cur, 1, M->corr, nullptr, RHS_NONE, M->nxt,
                                 nullptr, P->m));
        P->stats.fine_passes_fp64 += 1;
      } else {
        Group::check(M, P->copy_cpoints(0, 0, M->cur, 1, M->corr, M->nxt));
      }
    }
    G.flush(a);
    a = live(a);
    for (Member* M : a) {
      Plan* P = M->P;
      if (mixed) {
        // r = Phi^m d with d = v - (cur + corr) formed at the start
        Group::check(M, P->relax(0, 1, MODE_FC, M->nxt, 1, nullptr, nullptr, RHS_NONE,
                                 P->lev[0].R, P->partial, P->m, nullptr, M->cur, M->corr));
        P->stats.fine_passes_fp32 += 1;
      } else {
        Group::check(M, P->relax(0, 0, MODE_RES, M->nxt, 1, nullptr, nullptr, RHS_NONE,
                                 P->lev[0].R, P->partial, P->m));
        P->stats.fine_passes_fp64 += 1;
      }
    }
    G.flush(a);
    a = live(a);
    G.norms(a);
    for (Member* M : a)
      if (alive(M)) judge(M, M->it);
    a = live(a);
    correct(G, a, 0);
    for (Member* M : live(a)) {
      M->corr = M->P->lev[1].X;
      std::swap(M->cur, M->nxt);
      ++M->it;
    }
  }
  for (Member* M : all) {
    Plan* P = M->P;
    P->stats.iterations = M->it;
    if (mixed) P->stats.outer_iterations = M->it + 1;
    if (M->rc == MGRIT_OK) Group::check(M, finish_output(P, M->nxt, M->u_out, M->out_kind));
  }
  G.flush(all);
}

// F-relaxation (Parareal) with FP32 relaxation, as FP64 iterative
// refinement: the FP64 residual r of the iterate u, inner MGRIT cycles with
// FP32 relaxation on the error system e^{j+1} = Phi^m e^j + r^{j+1}
// (sequential coarse solve, residual subtraction and norms in FP64), then
// u += e in FP64.
void solve_ir(Group& G, const List& all) {
  const double kInnerDrop = 1e-5;  // inner solve target relative to |r|
  const int kInnerMax = 8;
  for (Member* M : all) Group::check(M, init_iterate(M->P, M->u0, M->uinit, M->P->U));
  for (;;) {
    List a = live(all);
    if (a.empty()) break;
    for (Member* M : a) {
      Plan* P = M->P;
      Group::check(M, P->relax(0, 0, MODE_RES, P->U, 1, nullptr, nullptr, RHS_NONE, P->Rout,
                               P->partial, P->m));
      P->stats.fine_passes_fp64 += 1;
    }
    G.flush(a);
    a = live(a);
    G.norms(a);
    for (Member* M : a)
      if (alive(M)) judge(M, M->it);
    a = live(a);
    for (Member* M : a) {
      M->cur = M->P->Va;
      M->nxt = M->P->Vb;
      M->corr = nullptr;
      M->prev = M->res;
      M->k = 0;
      M->inner = true;
    }
    const List outer = a;
    // inner cycles until each member's inner residual target
    for (;;) {
      List in;
      for (Member* M : live(outer))
        if (M->inner) in.push_back(M);
      if (in.empty()) break;
      for (Member* M : in) {
        Plan* P = M->P;
        const double* start = M->k == 0 ? nullptr : M->cur;
        if (P->relax_kind == MGRIT_RELAX_FCF) {
          Group::check(M, P->relax(0, 1, MODE_FC, start, 1, M->corr, P->Rout, RHS_CPOINT,
                                   M->nxt, nullptr, P->m));
          P->stats.fine_passes_fp32 += 1;
        } else {
          Group::check(M, P->copy_cpoints(0, 1, start, 1, M->corr, M->nxt));
        }
      }
      G.flush(in);
      in = live(in);
      for (Member* M : in) {
        Plan* P = M->P;
        Group::check(M, P->relax(0, 1, MODE_RES, M->nxt, 1, nullptr, P->Rout, RHS_CPOINT,
                                 P->lev[0].R, P->partial, P->m));
        P->stats.fine_passes_fp32 += 1;
      }
      G.flush(in);
      in = live(in);
      // the inner residual is kept apart from the outer one of M->res
      std::vector<double> outer_res(in.size());
      for (size_t i = 0; i < in.size(); ++i) outer_res[i] = in[i]->res;
      G.norms(in);
      List more;
      for (size_t i = 0; i < in.size(); ++i) {
        Member* M = in[i];
        const double rho = M->res;
        M->res = outer_res[i];
        if (!alive(M)) continue;
        if (!std::isfinite(rho)) {
          M->status = MGRIT_EDIVERGED;
          M->done = true;
          M->inner = false;
          continue;
        }
        // stop at the target, at the cap, or once a coarse correction stops
        // halving the inner residual (FP32 rounding floor)
        const bool stop = rho <= kInnerDrop * M->res || M->k + 1 >= kInnerMax ||
                          (M->k >= 1 && rho > 0.5 * M->prev);
        M->prev = rho;
        if (stop) M->inner = false;
        else more.push_back(M);
      }
      correct(G, more, 1);
      for (Member* M : live(more)) {
        ++M->inner_total;
        M->corr = M->P->lev[1].X;
        std::swap(M->cur, M->nxt);
        ++M->k;
      }
    }
    // u += e (the FCF-relaxed inner iterate whose residual was tested)
    for (Member* M : live(outer)) {
      Plan* P = M->P;
      const long long cells = (long long)(P->nt / P->m + 1) * P->nx;
      hipEvent_t e0 = nullptr;
      if (P->profiling) {
        P->tag = ProfTag();
        P->tag.pass = MGRIT_PASS_COPY;
        P->tag.bytes = 3.0 * cells * 8.0;
        P->tag.flops = (double)cells;
      }
      P->mark_util(MGRIT_PROF_OTHER, e0);
      launch_axpy(P->U, M->nxt, cells, G.stream());
      P->end_util(MGRIT_PROF_OTHER, e0);
      ++M->inner_total;
      ++M->it;
    }
  }
  for (Member* M : all) {
    Plan* P = M->P;
    P->stats.iterations = M->inner_total;
    P->stats.outer_iterations = M->it;
    if (M->rc == MGRIT_OK) Group::check(M, finish_output(P, P->U, M->u_out, M->out_kind));
  }
  G.flush(all);
}

}  // namespace

int solve_group(Plan* const* plans, int n, const double* const* u0, const double* const* uinit,
                const double* tol, const int* maxit, double* const* u_out, const int* out_kind,
                double* const* hist, int* iters, int* status) {
  if (n < 1) return MGRIT_EINVAL;
  const hipStream_t stream = plans[0]->stream;
  std::vector<Member> ms(n);
  List all;
  for (int i = 0; i < n; ++i) {
    Plan* P = plans[i];
    Member& M = ms[i];
    M.P = P;
    M.u0 = u0[i];
    M.uinit = uinit ? uinit[i] : nullptr;
    M.tol = tol[i];
    M.maxit = maxit[i];
    M.u_out = u_out ? u_out[i] : nullptr;
    M.out_kind = out_kind[i];
    M.hist = hist ? hist[i] : nullptr;
    std::memset(&P->stats, 0, sizeof P->stats);
    all.push_back(&M);
  }
  auto t0 = std::chrono::steady_clock::now();
  Group G(stream, n > 1);
  G.attach(all);
  // members of one solve form: FP64, FP32 with FCF (correction form), FP32
  // iterative refinement (F-relaxation, or asked for)
  List plain, mixed, ir;
  for (Member* M : all) {
    const Plan* P = M->P;
    if (P->precision == MGRIT_FP64) plain.push_back(M);
    else if (P->precision == MGRIT_FP32_RELAX && P->relax_kind == MGRIT_RELAX_FCF)
      mixed.push_back(M);
    else ir.push_back(M);
  }
  if (!plain.empty()) solve_plain(G, plain, false);
  if (!mixed.empty()) solve_plain(G, mixed, true);
  if (!ir.empty()) solve_ir(G, ir);
  G.detach(all);
  const bool synced = hipStreamSynchronize(stream) == hipSuccess;
  auto t1 = std::chrono::steady_clock::now();
  const double ms_all = std::chrono::duration<double, std::milli>(t1 - t0).count();
  int worst = MGRIT_OK;
  for (int i = 0; i < n; ++i) {
    Member& M = ms[i];
    if (!synced) Group::fail(&M, MGRIT_EHIP);
    M.P->stats.solve_ms = ms_all;
    if (iters) iters[i] = M.P->stats.iterations;
    status[i] = M.rc != MGRIT_OK ? M.rc : M.status;
    if (M.rc != MGRIT_OK && worst == MGRIT_OK) worst = M.rc;
  }
  return worst;
}

}  // namespace mgr

using namespace mgr;

extern "C" {

int mgrit_solve(mgrit_plan_t plan, const double* u0, const double* uinit, double tol,
                int maxit, double* u_out, int out_kind, double* hist, int* iters) {
  if (!plan || !u0 || maxit < 0 || !(tol >= 0.0)) return MGRIT_EINVAL;
  if (out_kind != MGRIT_OUT_NONE && !u_out) return MGRIT_EINVAL;
  if (out_kind < MGRIT_OUT_NONE || out_kind > MGRIT_OUT_ALL) return MGRIT_EINVAL;
  Plan* P = reinterpret_cast<Plan*>(plan);
  int status = MGRIT_OK;
  const int rc = solve_group(&P, 1, &u0, &uinit, &tol, &maxit, &u_out, &out_kind, &hist, iters,
                             &status);
  return rc ? rc : status;
}

int mgrit_solve_batch(int n, const mgrit_plan_t* plans, const double* const* u0,
                      const double* const* uinit, const double* tol, const int* maxit,
                      double* const* u_out, const int* out_kind, double* const* hist,
                      int* iters, int* status) {
  if (n < 1 || !plans || !u0 || !tol || !maxit || !out_kind || !status) return MGRIT_EINVAL;
  std::vector<Plan*> ps(n);
  for (int i = 0; i < n; ++i) {
    Plan* P = reinterpret_cast<Plan*>(plans[i]);
    if (!P || !u0[i] || maxit[i] < 0 || !(tol[i] >= 0.0)) return MGRIT_EINVAL;
    if (out_kind[i] < MGRIT_OUT_NONE || out_kind[i] > MGRIT_OUT_ALL) return MGRIT_EINVAL;
    if (out_kind[i] != MGRIT_OUT_NONE && (!u_out || !u_out[i])) return MGRIT_EINVAL;
    if (P->stream != reinterpret_cast<Plan*>(plans[0])->stream) return MGRIT_EINVAL;
    for (int k = 0; k < i; ++k)
      if (ps[k] == P) return MGRIT_EINVAL;  // a plan holds the state of one solve
    ps[i] = P;
  }
  return solve_group(ps.data(), n, u0, uinit, tol, maxit, u_out, out_kind, hist, iters, status);
}

}  // extern "C"
