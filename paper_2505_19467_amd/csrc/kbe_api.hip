// Context and C ABI (include/kbe.h) of the gfx950 Kadanoff-Baym library: workspace
// layout over caller-owned device buffers, and the per-step launch sequence of
// Algorithm "prop" (predictor, K corrector passes, evaluation on the accepted row).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kbe.h"
#include "kbe_adjoint.hpp"
#include "kbe_kernels.hpp"

using kbe::cplx;
using kbe::Dims;
using kbe::LaunchArgs;

namespace {

enum {
  B_SIGMA = 0, B_IA, B_IB, B_RHOA, B_RHOB, B_DA, B_DB, B_PROP, B_COL0, B_DIAG, B_COLSUM, B_ROWPART,
  B_HF, B_HOP, B_EIGW, B_EIGU, B_MU, B_ROW64, B_CHG, B_CHGMAX, B_GR, B_COUNT
};

struct Layout {
  Dims d;
  size_t off[B_COUNT];
  size_t bytes[B_COUNT];
  size_t ws_bytes, hist_bytes, obs_bytes;
};

int make_layout(const kbe_config* c, Layout* L, std::string* why) {
  if (!c) { *why = "null config"; return KBE_ERR_INVALID_ARG; }
  if (c->nb < 1 || c->nb > 4) { *why = "nb must be 1..4"; return KBE_ERR_SHAPE; }
  // a 1D chain (nky = 1) up to 1024 k-points, a 2D grid up to 64 per axis; N_k <= 1024 keeps the
  // self-energy kernels' LDS tile (four lines and the roots of unity) within 82 KB
  if (c->nkx < 1 || c->nky < 1 || c->nkx * c->nky > 1024 || (c->nky > 1 && (c->nkx > 64 || c->nky > 64))) {
    *why = "k grid must be a chain of 1..1024 points (nky = 1) or a 2D grid with nkx, nky <= 64 and nkx * nky <= 1024";
    return KBE_ERR_SHAPE;
  }
  if (c->nt_max < 1 || c->nt_max > 8192) { *why = "nt_max must be 1..8192"; return KBE_ERR_SHAPE; }
  if (c->interaction != KBE_INT_HUBBARD && c->interaction != KBE_INT_INTERBAND) {
    *why = "interaction must be KBE_INT_HUBBARD or KBE_INT_INTERBAND";
    return KBE_ERR_INVALID_ARG;
  }
  if (c->interaction == KBE_INT_INTERBAND && c->nb != 2) { *why = "the interband preset needs nb = 2"; return KBE_ERR_SHAPE; }
  if (c->precision != KBE_FP64 && c->precision != KBE_FP32 && c->precision != KBE_FP32_MFMA) {
    *why = "precision must be KBE_FP64, KBE_FP32 or KBE_FP32_MFMA";
    return KBE_ERR_INVALID_ARG;
  }
  if (c->n_corr < 0 || c->n_corr > 16) { *why = "n_corr must be 0..16"; return KBE_ERR_INVALID_ARG; }
  if (!(c->corr_tol >= 0.0) || !std::isfinite(c->corr_tol)) { *why = "corr_tol must be finite and >= 0"; return KBE_ERR_INVALID_ARG; }
  if (c->corr_tol > 0.0 && c->n_corr < 1) { *why = "corr_tol > 0 needs n_corr >= 1 (the most passes)"; return KBE_ERR_INVALID_ARG; }
  if (c->quad_points < 0 || c->quad_points > kbe::KBE_QMAX) { *why = "quad_points must be 0..6 (0 or 1: trapezoid)"; return KBE_ERR_INVALID_ARG; }
  if (!(c->dt > 0.0) || !(c->temp > 0.0) || !std::isfinite(c->U) || c->spin_deg < 1 || c->spin_deg > 2) {
    *why = "dt and temp must be positive, U finite, spin_deg 1 or 2";
    return KBE_ERR_INVALID_ARG;
  }
  Dims& d = L->d;
  d.nkx = c->nkx;
  d.nky = c->nky;
  d.nk = c->nkx * c->nky;
  d.nb = c->nb;
  d.nbb = c->nb * c->nb;
  d.C = 2 * d.nbb;
  d.Tp = ((c->nt_max + 1 + 7) / 8) * 8;
  d.Smax = (c->nt_max + 63) / 64;
  d.fp32 = c->precision == KBE_FP64 ? 0 : 1;
  d.mfma = c->precision == KBE_FP32_MFMA ? 1 : 0;
  d.spb = (c->nb <= 2 && !d.mfma) ? 2 : 1;
  d.qp = c->quad_points > 1 ? c->quad_points : 1;
  d.rring = d.qp > 2 ? d.qp : 2;
  d.N = c->nt_max + 1;
  d.P = d.mfma ? 256 * kbe::quad_base((d.N + 63) / 64, d.N) : kbe::strip_base((d.N + 63) / 64, d.N);
  const size_t cz = sizeof(cplx);
  size_t nk = d.nk;
  size_t sz[B_COUNT];
  sz[B_SIGMA] = nk * 3 * d.nbb * d.Tp * cz;
  sz[B_IA] = sz[B_IB] = nk * d.C * d.Tp * cz;
  sz[B_RHOA] = sz[B_RHOB] = sz[B_DA] = sz[B_DB] = nk * d.nbb * cz;
  sz[B_PROP] = nk * 3 * d.nbb * cz;
  sz[B_COLSUM] = nk * d.C * d.Tp * cz;
  sz[B_COL0] = sz[B_DIAG] = nk * d.C * (size_t)d.qp * d.Tp * cz;  // qp columns / band offsets
  sz[B_ROWPART] = nk * (size_t)d.Smax * d.nbb * d.Tp * cz;
  sz[B_HF] = d.nbb * cz;
  sz[B_HOP] = 3 * d.nbb * cz;
  sz[B_EIGW] = nk * d.nb * sizeof(double);
  sz[B_EIGU] = nk * d.nbb * cz;
  sz[B_MU] = sizeof(double);
  sz[B_ROW64] = (size_t)d.rring * nk * d.C * d.Tp * cz;
  // corrector change per (k, t') and its maximum, only when the corrector stops on a tolerance
  sz[B_CHG] = c->corr_tol > 0.0 ? nk * d.Tp * sizeof(double) : 0;
  sz[B_CHGMAX] = c->corr_tol > 0.0 ? sizeof(double) : 0;
  // interband self-energy: real-space lines of the current row, [t_j][comp][ab][R]
  sz[B_GR] = c->interaction == KBE_INT_INTERBAND ? (size_t)d.Tp * 2 * d.nbb * nk * cz : 0;
  size_t off = 0;
  for (int i = 0; i < B_COUNT; ++i) {
    L->off[i] = off;
    L->bytes[i] = sz[i];
    off += (sz[i] + 255) / 256 * 256;
  }
  L->ws_bytes = off;
  L->hist_bytes = (size_t)nk * d.C * (size_t)d.P * (d.fp32 ? sizeof(float2) : cz);
  L->obs_bytes = (size_t)(c->nt_max + 1) * KBE_NOBS * sizeof(double);
  return KBE_OK;
}

// End corrections of the collision-integral quadrature for q = 1..qp nodes per end. The
// trapezoid sum of a polynomial differs from its integral by end terms only
// (Euler-Maclaurin); corrections c_0..c_{q-1} on the first q nodes cancel the left end's
// terms for every polynomial of degree < q, i.e. for f = x^d the moments
//   sum_{j<q} c_j j^d = -1/2 [d = 0] + [d odd] B_{d+1} / (d + 1),  d = 0..q-1,
// with B_n the Bernoulli numbers (generating function x / (e^x - 1)). Solved here by
// Gauss-Jordan elimination; q = 1 gives the trapezoid's -1/2.
kbe::QuadW quad_corrections(int qp) {
  kbe::QuadW Q{};
  Q.q = qp;
  // Bernoulli numbers from B_n = -1/(n+1) sum_{k<n} binom(n+1, k) B_k
  double B[kbe::KBE_QMAX + 2] = {1.0};
  for (int n = 1; n <= kbe::KBE_QMAX + 1; ++n) {
    double acc = 0.0, binom = 1.0;
    for (int k = 0; k < n; ++k) {
      acc += binom * B[k];
      binom *= (double)(n + 1 - k) / (double)(k + 1);
    }
    B[n] = -acc / (n + 1);
  }
  for (int q = 1; q <= qp; ++q) {
    double M[kbe::KBE_QMAX][kbe::KBE_QMAX + 1];
    for (int row = 0; row < q; ++row) {
      double pw = 1.0;  // j^row, 0^0 = 1
      for (int j = 0; j < q; ++j) {
        pw = 1.0;
        for (int e = 0; e < row; ++e) pw *= j;
        M[row][j] = pw;
      }
      M[row][q] = (row == 0 ? -0.5 : 0.0) + (row % 2 == 1 ? B[row + 1] / (row + 1) : 0.0);
    }
    for (int col = 0; col < q; ++col) {
      int best = col;
      for (int r = col + 1; r < q; ++r)
        if (std::fabs(M[r][col]) > std::fabs(M[best][col])) best = r;
      if (best != col)
        for (int x = 0; x <= q; ++x) std::swap(M[col][x], M[best][x]);
      for (int r = 0; r < q; ++r) {
        if (r == col) continue;
        double f = M[r][col] / M[col][col];
        for (int x = col; x <= q; ++x) M[r][x] -= f * M[col][x];
      }
    }
    for (int j = 0; j < q; ++j) Q.c[q][j] = M[j][q] / M[j][j];
  }
  return Q;
}

double pulse_A(const kbe_pulse& p, double t) {
  if (p.kind != KBE_PULSE_PEIERLS || p.width <= 0.0) return 0.0;
  double x = (t - p.t0) / p.width;
  return p.amp * std::sin(p.omega * t) * std::exp(-x * x);
}
// dA/d(amp) and dA/d(omega) at t
void pulse_dA(const kbe_pulse& p, double t, double* damp, double* domega) {
  *damp = *domega = 0.0;
  if (p.kind != KBE_PULSE_PEIERLS || p.width <= 0.0) return;
  double x = (t - p.t0) / p.width;
  double g = std::exp(-x * x);
  *damp = std::sin(p.omega * t) * g;
  *domega = p.amp * t * std::cos(p.omega * t) * g;
}

// Adjoint workspace: adjoint history + per-step rows of the reverse sweep.
enum {
  A_LAM = 0, A_IBAR0, A_IBAR1, A_IBARC, A_RBAR, A_SBAR, A_SBARCOL, A_IREPREV, A_IREC, A_SBARRP,
  A_DBAR0, A_DBAR1, A_DBARC, A_RHOBAR0, A_RHOBAR1, A_RHOBARP, A_RHOP, A_DC, A_DSCR, A_RHO0,
  A_PROPSP, A_PROPSC, A_PBAR, A_HFP, A_HFC, A_KPART, A_UBAR, A_THETA, A_SIGEV, A_COUNT
};

size_t adj_layout(const Layout& L, size_t* off) {
  const Dims& d = L.d;
  const size_t cz = sizeof(cplx), nk = d.nk;
  size_t sz[A_COUNT];
  sz[A_LAM] = nk * d.C * (size_t)d.P * cz;
  size_t row = nk * d.C * d.Tp * cz;
  for (int i = A_IBAR0; i <= A_IREC; ++i) sz[i] = row;
  sz[A_SBARRP] = nk * (size_t)d.Smax * d.nbb * d.Tp * cz;
  size_t mat = nk * d.nbb * cz;
  for (int i = A_DBAR0; i <= A_RHO0; ++i) sz[i] = mat;
  sz[A_PROPSP] = sz[A_PROPSC] = sz[A_PBAR] = 3 * mat;
  sz[A_HFP] = sz[A_HFC] = d.nbb * cz;
  sz[A_KPART] = nk * (d.nb + 1) * sizeof(double);
  sz[A_UBAR] = ((size_t)((d.N * d.nbb + 7) / 8) * 8) * sizeof(double);
  sz[A_THETA] = 3 * sizeof(double);
  sz[A_SIGEV] = nk * 3 * d.nbb * d.Tp * cz;   // Sigma row of the evaluation pass, kept for the fused pass
  size_t o = 0;
  for (int i = 0; i < A_COUNT; ++i) {
    if (off) off[i] = o;
    o += (sz[i] + 255) / 256 * 256;
  }
  return o;
}

}  // namespace

struct kbe_ctx {
  kbe_config cfg;
  kbe_pulse pulse;
  Layout L;
  hipStream_t st;
  char* ws;
  void* hist;
  double* obs;
  int cur;   // slot holding the *_prev role
  int step;  // last completed step
  std::string err;
  std::vector<cplx> hop_host;
  // timing of the history-sum launches
  bool timing;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_m;
  size_t ev_used;
  // reverse sweep
  char* adj;
  size_t adj_off[A_COUNT];
  int adj_obs;   // observable of the sweep (-1: not started)
  int adj_m;     // next step to reverse
  int adj_cur;   // role of the double-buffered adjoint rows
  bool frozen;   // working buffers overwritten by a reverse sweep
  kbe::QuadW quad;  // end corrections of the collision-integral quadrature
  // corrector log (host): passes taken per step, and the row change after each pass
  std::vector<int32_t> passes;
  std::vector<double> changes;
  int noalloc_dev = -1;  // device whose static workspace this context holds (kbe_create_noalloc)

  template <class T>
  T* buf(int b) const { return reinterpret_cast<T*>(ws + L.off[b]); }

  LaunchArgs args() const {
    LaunchArgs a;
    a.hist = hist;
    a.row64 = buf<cplx>(B_ROW64);
    a.sig = buf<cplx>(B_SIGMA);
    a.I_prev = buf<cplx>(cur == 0 ? B_IA : B_IB);
    a.I_cur = buf<cplx>(cur == 0 ? B_IB : B_IA);
    a.col0 = buf<cplx>(B_COL0);
    a.diag = buf<cplx>(B_DIAG);
    a.colsum = buf<cplx>(B_COLSUM);
    a.rowpart = buf<cplx>(B_ROWPART);
    a.rho_prev = buf<cplx>(cur == 0 ? B_RHOA : B_RHOB);
    a.rho_cur = buf<cplx>(cur == 0 ? B_RHOB : B_RHOA);
    a.D_prev = buf<cplx>(cur == 0 ? B_DA : B_DB);
    a.D_cur = buf<cplx>(cur == 0 ? B_DB : B_DA);
    a.props = buf<cplx>(B_PROP);
    a.hfbuf = buf<cplx>(B_HF);
    a.hop = buf<cplx>(B_HOP);
    a.eig_w = buf<double>(B_EIGW);
    a.eig_U = buf<cplx>(B_EIGU);
    a.mu = buf<double>(B_MU);
    a.obs = obs;
    a.commit = 1;
    a.chg = nullptr;
    a.gR = L.bytes[B_GR] ? buf<cplx>(B_GR) : nullptr;
    a.quad = quad;
    a.Ax = a.Ay = 0.0;
    a.polx = pulse.pol[0];
    a.poly = pulse.pol[1];
    a.dt = cfg.dt;
    a.U = cfg.U;
    a.UU = cfg.U * cfg.U;
    a.temp = cfg.temp;
    a.target = (double)cfg.nb * cfg.filling * (double)L.d.nk;
    a.spin = cfg.spin_deg;
    a.interaction = cfg.interaction;
    a.hf = cfg.hf;
    a.corr = cfg.corr;
    return a;
  }
  void set_A(LaunchArgs& a, double t) const {
    double A = pulse_A(pulse, t);
    a.Ax = A * pulse.pol[0];
    a.Ay = A * pulse.pol[1];
  }
  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
  int check(hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(KBE_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return KBE_OK;
  }
  int bulk_timed(const LaunchArgs& a, int m) {
    // the event pool is created whole by kbe_timing before any launch is queued; launches past
    // its end (more passes than it was sized for) run untimed
    if (timing && m >= 1 && ev_used + 2 <= ev.size()) {
      if (hipEventRecord(ev[ev_used], st) != hipSuccess) return fail(KBE_ERR_HIP, "hipEventRecord failed");
      int rc = check(kbe::launch_bulk(L.d, a, m, st), "history-sum launch");
      if (rc) return rc;
      if (hipEventRecord(ev[ev_used + 1], st) != hipSuccess) return fail(KBE_ERR_HIP, "hipEventRecord failed");
      ev_used += 2;
      ev_m.push_back(m);
    } else {
      int rc = check(kbe::launch_bulk(L.d, a, m, st), "history-sum launch");
      if (rc) return rc;
    }
    return check(kbe::launch_rowpart_fold(L.d, a, m, st), "row-partial fold launch");
  }
  // Sigma row, equal-time collision integral, history sums of row m.
  int collision_parts(LaunchArgs& a, int m) {
    int rc = check(kbe::launch_sigma(L.d, a, m, st), "self-energy launch");
    if (!rc) rc = check(kbe::launch_diag_I(L.d, a, m, st), "equal-time collision launch");
    if (!rc) rc = bulk_timed(a, m);
    return rc;
  }
  // The dipole pulse E(t) = I delta(t - t0) of eq. (dipole) acts as the kick K = exp(-i I X) on the
  // slice at the grid time t_{m0} nearest t0 (m0 = floor(t0 / dt + 1/2)): once the slice is
  // complete (its observables are the values just before the kick) the row and rho_m0 are
  // kicked and the slice's self-energy and collision integrals are evaluated again on the kicked
  // row; they feed the next step's predictor (at m0 = 0 the integrals are empty).
  int kick_slice() const { return (int)std::floor(pulse.t0 / cfg.dt + 0.5); }
  int dipole_kick(int m) {
    if (pulse.kind != KBE_PULSE_DIPOLE_KICK || m != kick_slice()) return KBE_OK;
    LaunchArgs a = args();
    int rc = check(kbe::launch_kick(L.d, a, m, std::cos(pulse.amp), std::sin(pulse.amp),
                                    m == 0 ? a.rho_prev : a.rho_cur, st),
                   "dipole-kick launch");
    if (!rc && m > 0) rc = collision_parts(a, m);
    if (!rc && m > 0) rc = check(kbe::launch_row(L.d, a, m, KBE_ROW_EVAL, st), "collision-row launch");
    return rc;
  }
  int props(LaunchArgs& a, int m, int mode) {
    set_A(a, (m - 0.5) * cfg.dt);
    int rc = check(kbe::launch_hf(L.d, a, mode == 0 ? 0.0 : 0.5, st), "mean-field launch");
    if (!rc) rc = check(kbe::launch_props(L.d, a, st), "propagator launch");
    return rc;
  }
  int observe(int m) {
    LaunchArgs a = args();
    double t = m * cfg.dt;
    set_A(a, t);
    return check(kbe::launch_obs(L.d, a, m, t, pulse_A(pulse, t), st), "observables launch");
  }
  int one_step() {
    int m = step + 1;
    if (m > cfg.nt_max) return fail(KBE_ERR_STATE, "step index would pass nt_max");
    LaunchArgs a = args();
    int rc = props(a, m, 0);
    if (!rc) rc = check(kbe::launch_row(L.d, a, m, KBE_ROW_PREDICT, st), "predictor launch");
    // Corrector passes of Algorithm "prop": all n_corr of them, or (corr_tol > 0) until the
    // largest change of row m is <= corr_tol, which needs the change on the host after each
    // pass (one stream synchronisation per pass in that mode).
    const bool tol = cfg.corr_tol > 0.0;
    bool reached = !tol;
    double last_change = 0.0;
    int taken = 0;
    for (int it = 0; it < cfg.n_corr && !rc; ++it) {
      rc = collision_parts(a, m);
      if (!rc) rc = props(a, m, 1);
      a.chg = tol ? buf<double>(B_CHG) : nullptr;
      if (!rc) rc = check(kbe::launch_row(L.d, a, m, KBE_ROW_CORRECT, st), "corrector launch");
      a.chg = nullptr;
      if (rc) break;
      ++taken;
      if (tol) {
        double ch = 0.0;
        rc = check(kbe::launch_change_max(L.d, buf<double>(B_CHG), m, buf<double>(B_CHGMAX), st),
                   "corrector change launch");
        if (!rc)
          rc = check(hipMemcpyAsync(&ch, buf<double>(B_CHGMAX), sizeof(double), hipMemcpyDeviceToHost, st),
                     "corrector change copy");
        if (!rc) rc = check(hipStreamSynchronize(st), "stream synchronisation");
        if (rc) break;
        if (!std::isfinite(ch)) {
          rc = fail(KBE_ERR_NONFINITE, "non-finite corrector change");
          break;
        }
        changes[(size_t)m * cfg.n_corr + it] = ch;
        last_change = ch;
        if (ch <= cfg.corr_tol) {
          reached = true;
          break;
        }
      }
    }
    if (!rc) passes[m] = taken;
    if (!rc) rc = collision_parts(a, m);
    if (!rc) rc = check(kbe::launch_row(L.d, a, m, KBE_ROW_EVAL, st), "collision-row launch");
    if (!rc) rc = observe(m);
    if (!rc) rc = dipole_kick(m);
    if (rc) return rc;
    cur ^= 1;
    step = m;
    // Algorithm "prop" left its corrector loop on the pass limit without reaching epsilon: the
    // step is committed (as the algorithm proceeds) and reported to the caller
    if (!reached && cfg.n_corr > 0)
      return fail(KBE_ERR_NOT_CONVERGED, "step " + std::to_string(m) + ": the row still changed by " +
                                             std::to_string(last_change) + " after " + std::to_string(taken) +
                                             " corrector passes (corr_tol " + std::to_string(cfg.corr_tol) + ")");
    return KBE_OK;
  }

  // ---------------------------------------------------------------- reverse sweep
  template <class T>
  T* abuf(int i) const { return reinterpret_cast<T*>(adj + adj_off[i]); }
  kbe::AdjArgs adj_args() const {
    kbe::AdjArgs b;
    int c = adj_cur;
    b.lam = abuf<cplx>(A_LAM);
    b.Ibar = abuf<cplx>(c == 0 ? A_IBAR0 : A_IBAR1);
    b.Ibar_prev = abuf<cplx>(c == 0 ? A_IBAR1 : A_IBAR0);
    b.Ibar_c = abuf<cplx>(A_IBARC);
    b.Rbar = abuf<cplx>(A_RBAR);
    b.sbar = abuf<cplx>(A_SBAR);
    b.sbar_col = abuf<cplx>(A_SBARCOL);
    b.sbar_rowpart = abuf<cplx>(A_SBARRP);
    b.Dbar = abuf<cplx>(c == 0 ? A_DBAR0 : A_DBAR1);
    b.Dbar_prev = abuf<cplx>(c == 0 ? A_DBAR1 : A_DBAR0);
    b.Dbar_c = abuf<cplx>(A_DBARC);
    b.rhobar = abuf<cplx>(c == 0 ? A_RHOBAR0 : A_RHOBAR1);
    b.rhobar_prev = abuf<cplx>(c == 0 ? A_RHOBAR1 : A_RHOBAR0);
    b.rhobar_P = abuf<cplx>(A_RHOBARP);
    b.props_p = abuf<cplx>(A_PROPSP);
    b.props_c = abuf<cplx>(A_PROPSC);
    b.pbar = abuf<cplx>(A_PBAR);
    b.rhoP = abuf<cplx>(A_RHOP);
    b.Ire_prev = abuf<cplx>(A_IREPREV);
    b.Ire_c = abuf<cplx>(A_IREC);
    b.Dc = abuf<cplx>(A_DC);
    b.Dscratch = abuf<cplx>(A_DSCR);
    b.rho0 = abuf<cplx>(A_RHO0);
    b.hf_p = abuf<cplx>(A_HFP);
    b.hf_c = abuf<cplx>(A_HFC);
    b.kpart = abuf<double>(A_KPART);
    b.ubar_part = abuf<double>(A_UBAR);
    b.theta_bar = abuf<double>(A_THETA);
    return b;
  }
  int zero_adj(int i, size_t bytes) {
    return check(kbe::launch_fill_zero(abuf<double>(i), (int64_t)(bytes / sizeof(double)), st), "zero");
  }
  int adj_seed(int obs_id) {
    const Dims& d = L.d;
    size_t row = (size_t)d.nk * d.C * d.Tp * sizeof(cplx), mat = (size_t)d.nk * d.nbb * sizeof(cplx);
    int rc = zero_adj(A_LAM, (size_t)d.nk * d.C * (size_t)d.P * sizeof(cplx));
    for (int i = A_IBAR0; i <= A_IBAR1 && !rc; ++i) rc = zero_adj(i, row);
    // A_RHOP too: the recomputed predictor's mean field reads it with weight 0 before it is written
    for (int i = A_DBAR0; i <= A_RHOP && !rc; ++i) rc = zero_adj(i, mat);
    if (!rc) rc = zero_adj(A_THETA, 3 * sizeof(double));
    if (rc) return rc;
    LaunchArgs a = args();
    double T = step * cfg.dt, damp, dom;
    set_A(a, T);
    pulse_dA(pulse, T, &damp, &dom);
    kbe::AdjArgs b = adj_args();
    rc = check(kbe::launch_adj_rho(d, hist, step, b.rho0, st), "density read-back launch");
    if (!rc) rc = check(kbe::launch_adj_seed(d, a, b, b.rho0, obs_id, damp, dom, st), "adjoint seed launch");
    return rc;
  }
  int adj_sigma_pass(const LaunchArgs& a, const kbe::AdjArgs& b, const cplx* Ibar, const cplx* Dbar, int m,
                     int mode, const cplx* sig1 = nullptr, const cplx* Ibar1 = nullptr) {
    const Dims& d = L.d;
    int nblk = 0;
    int rc = check(kbe::launch_adj_bulk(d, a, b, Ibar, m, mode, sig1, Ibar1, st), "adjoint history-sum launch");
    if (!rc) rc = check(kbe::launch_adj_row(d, a, b, Ibar, Dbar, m, st), "adjoint end-point launch");
    if (!rc) rc = check(kbe::launch_adj_sigma(d, a, b, m, &nblk, st), "adjoint self-energy launch");
    if (!rc) rc = check(kbe::launch_adj_reduce_u(b, nblk, st), "adjoint reduction launch");
    return rc;
  }
  // Reverse step m (t_m -> t_{m-1}) of the K = 1 scheme: evaluation pass, corrector
  // update, corrector mean field/propagators, corrector collision pass, predictor update,
  // predictor mean field/propagators.
  int adj_reverse(int m) {
    const Dims& d = L.d;
    LaunchArgs a = args();
    double tm = (m - 0.5) * cfg.dt, damp, dom;
    set_A(a, tm);
    pulse_dA(pulse, tm, &damp, &dom);
    kbe::AdjArgs b = adj_args();
    // The committed history is every time slice's checkpoint: rho_{m-1} is its diagonal block,
    // and D_{m-1} comes out of the recomputed evaluation pass of t_{m-1} below.
    cplx* rho0 = b.rho0;
    int rc = check(kbe::launch_adj_rho(d, hist, m - 1, rho0, st), "density read-back launch");
    // committed rows m-1, m, column 0 and diagonal
    if (!rc) rc = check(kbe::launch_aux(d, a, m, st), "aux launch");
    // Sigma of the committed row m, in a buffer of its own: the corrector pass below applies this
    // pass's adjoint-history update too (both updates are linear in their Sigma row and Ibar and
    // touch the same stored blocks), so the history and the adjoint history stream once for both
    LaunchArgs ev = a;
    ev.sig = abuf<cplx>(A_SIGEV);
    if (!rc) rc = check(kbe::launch_sigma(d, ev, m, st), "self-energy launch");
    // evaluation pass of t_m: Sigma adjoints only
    if (!rc) rc = adj_sigma_pass(ev, b, b.Ibar, b.Dbar, m, kbe::ADJ_SUMS);
    // recompute I(t_{m-1}, .)
    LaunchArgs e = a;
    e.I_cur = b.Ire_prev;
    e.D_cur = b.Dscratch;
    if (!rc) rc = check(kbe::launch_sigma(d, e, m - 1, st), "self-energy launch");
    if (!rc) rc = check(kbe::launch_diag_I(d, e, m - 1, st), "equal-time collision launch");
    if (!rc) rc = check(kbe::launch_bulk(d, e, m - 1, st), "history-sum launch");
    if (!rc) rc = check(kbe::launch_rowpart_fold(d, e, m - 1, st), "row-partial fold launch");
    if (!rc) rc = check(kbe::launch_row(d, e, m - 1, KBE_ROW_EVAL, st), "collision-row launch");
    // recompute the predictor (row m of the working copy only)
    LaunchArgs p = a;
    p.I_prev = b.Ire_prev;
    p.rho_prev = rho0;
    p.rho_cur = b.rhoP;
    p.D_prev = b.Dscratch;
    p.props = b.props_p;
    p.hfbuf = b.hf_p;
    p.commit = 0;
    if (!rc) rc = check(kbe::launch_hf(d, p, 0.0, st), "mean-field launch");
    if (!rc) rc = check(kbe::launch_props(d, p, st), "propagator launch");
    if (!rc) rc = check(kbe::launch_row(d, p, m, KBE_ROW_PREDICT, st), "predictor launch");
    // recompute the corrector's collision row and propagators
    LaunchArgs c = p;
    c.I_cur = b.Ire_c;
    c.D_cur = b.Dc;
    c.props = b.props_c;
    c.hfbuf = b.hf_c;
    if (!rc) rc = check(kbe::launch_sigma(d, c, m, st), "self-energy launch");
    if (!rc) rc = check(kbe::launch_diag_I(d, c, m, st), "equal-time collision launch");
    if (!rc) rc = check(kbe::launch_bulk(d, c, m, st), "history-sum launch");
    if (!rc) rc = check(kbe::launch_rowpart_fold(d, c, m, st), "row-partial fold launch");
    if (!rc) rc = check(kbe::launch_row(d, c, m, KBE_ROW_EVAL, st), "collision-row launch");
    if (!rc) rc = check(kbe::launch_hf(d, c, 0.5, st), "mean-field launch");
    if (!rc) rc = check(kbe::launch_props(d, c, st), "propagator launch");
    // corrector update, its propagators and mean field
    if (!rc) rc = check(kbe::launch_adj_update(d, p, b, m, 1, b.lam, b.Rbar, rho0, st), "adjoint update launch");
    if (!rc) rc = check(kbe::launch_adj_props(d, a, b, b.hf_c, st), "adjoint propagator launch");
    if (!rc)
      rc = check(kbe::launch_adj_hf(d, a, b, rho0, b.rhoP, 0.5, b.rhobar_prev, b.rhobar_P, damp, dom, st),
                 "adjoint mean-field launch");
    // corrector collision pass (Sigma of the predictor row, still in place)
    if (!rc) rc = adj_sigma_pass(a, b, b.Ibar_c, b.Dbar_c, m, kbe::ADJ_FUSED, ev.sig, b.Ibar);
    // predictor update, its propagators and mean field
    if (!rc) rc = check(kbe::launch_adj_update(d, p, b, m, 0, nullptr, b.Rbar, rho0, st), "adjoint update launch");
    if (!rc) rc = check(kbe::launch_adj_props(d, a, b, b.hf_p, st), "adjoint propagator launch");
    if (!rc)
      rc = check(kbe::launch_adj_hf(d, a, b, rho0, rho0, 0.0, b.rhobar_prev, nullptr, damp, dom, st),
                 "adjoint mean-field launch");
    if (rc) return rc;
    // the accumulated adjoints of step m-1 become the inputs of the next reverse step
    adj_cur ^= 1;
    size_t row = (size_t)d.nk * d.C * d.Tp * sizeof(cplx), mat = (size_t)d.nk * d.nbb * sizeof(cplx);
    rc = zero_adj(adj_cur == 0 ? A_IBAR1 : A_IBAR0, row);
    if (!rc) rc = zero_adj(adj_cur == 0 ? A_DBAR1 : A_DBAR0, mat);
    if (!rc) rc = zero_adj(adj_cur == 0 ? A_RHOBAR1 : A_RHOBAR0, mat);
    if (!rc) rc = zero_adj(A_RHOBARP, mat);
    return rc;
  }
};

namespace {

// kbe_create on the given workspace; clear_workspace zeroes all of it first (a workspace that
// keeps an earlier context's contents).
int create_context(const kbe_config* cfg, const double* hop, const kbe_pulse* pulse, void* d_history,
                   size_t history_bytes, void* d_workspace, size_t workspace_bytes, void* d_obs, size_t obs_bytes,
                   void* hip_stream, kbe_ctx** out, bool clear_workspace) {
  if (!out) return KBE_ERR_INVALID_ARG;
  *out = nullptr;
  if (!cfg || !hop || !d_history || !d_workspace || !d_obs) return KBE_ERR_INVALID_ARG;
  kbe_ctx* c = new kbe_ctx();
  c->cfg = *cfg;
  if (pulse) c->pulse = *pulse;
  else std::memset(&c->pulse, 0, sizeof(c->pulse));
  const kbe_pulse& pu = c->pulse;
  if ((pu.kind != KBE_PULSE_PEIERLS && pu.kind != KBE_PULSE_DIPOLE_KICK) ||
      (pu.kind == KBE_PULSE_DIPOLE_KICK && (cfg->nb != 2 || !(pu.t0 >= 0.0) || !std::isfinite(pu.amp) ||
                                            !std::isfinite(pu.t0)))) {
    delete c;
    return KBE_ERR_INVALID_ARG;
  }
  std::string why;
  int rc = make_layout(cfg, &c->L, &why);
  if (rc) {
    delete c;
    return rc;
  }
  if (history_bytes < c->L.hist_bytes || workspace_bytes < c->L.ws_bytes || obs_bytes < c->L.obs_bytes) {
    delete c;
    return KBE_ERR_INVALID_ARG;
  }
  c->st = (hipStream_t)hip_stream;
  c->ws = (char*)d_workspace;
  c->hist = d_history;
  c->obs = (double*)d_obs;
  c->cur = 0;
  c->step = 0;
  c->timing = false;
  c->ev_used = 0;
  c->adj = nullptr;
  c->adj_obs = -1;
  c->adj_m = 0;
  c->adj_cur = 0;
  c->frozen = false;
  c->quad = quad_corrections(c->L.d.qp);
  c->passes.assign((size_t)cfg->nt_max + 1, 0);
  c->changes.assign((size_t)(cfg->nt_max + 1) * (cfg->n_corr > 0 ? cfg->n_corr : 1), -1.0);
  const Dims& d = c->L.d;
  c->hop_host.resize(3 * d.nbb);
  for (int i = 0; i < 3 * d.nbb; ++i) c->hop_host[i] = make_double2(hop[2 * i], hop[2 * i + 1]);
  if (d.nky == 1)
    for (int i = 0; i < d.nbb; ++i) c->hop_host[2 * d.nbb + i] = make_double2(0.0, 0.0);
  LaunchArgs a = c->args();
  if (clear_workspace)
    rc = c->check(kbe::launch_fill_zero((double*)c->ws, c->L.ws_bytes / sizeof(double), c->st), "zero");
  if (!rc)
    rc = c->check(hipMemcpyAsync(a.hop, c->hop_host.data(), 3 * d.nbb * sizeof(cplx), hipMemcpyHostToDevice, c->st),
                  "copy of the hopping blocks");
  if (!rc) rc = c->check(kbe::launch_fill_zero((double*)c->buf<cplx>(B_IA), 2 * c->L.bytes[B_IA] / sizeof(cplx), c->st), "zero");
  if (!rc) rc = c->check(kbe::launch_fill_zero((double*)c->buf<cplx>(B_IB), 2 * c->L.bytes[B_IB] / sizeof(cplx), c->st), "zero");
  if (!rc) rc = c->check(kbe::launch_fill_zero((double*)c->buf<cplx>(B_DA), 2 * c->L.bytes[B_DA] / sizeof(cplx), c->st), "zero");
  if (!rc) rc = c->check(kbe::launch_fill_zero((double*)c->buf<cplx>(B_DB), 2 * c->L.bytes[B_DB] / sizeof(cplx), c->st), "zero");
  if (!rc) rc = c->check(kbe::launch_fill_zero(c->obs, c->L.obs_bytes / sizeof(double), c->st), "zero");
  if (!rc) {
    c->set_A(a, 0.0);
    rc = c->check(kbe::launch_init(d, a, c->st), "initial-state launch");
  }
  if (!rc) rc = c->observe(0);
  if (!rc) rc = c->dipole_kick(0);
  if (!rc) rc = c->check(hipStreamSynchronize(c->st), "initial state");
  if (rc) {
    delete c;
    return rc;
  }
  *out = c;
  return KBE_OK;
}

// ---------------------------------------------------------------- allocation-free contexts
// The workspace of a context made by kbe_create_noalloc: one array per device, loaded with the
// library's code and kept until the process ends. Host code never passes the array's name to a
// kernel or a copy (on the host it only stands for the symbol): it uses the device address
// that hipGetSymbolAddress returns for the current device, kept per device below.
constexpr size_t NOALLOC_BYTES = KBE_NOALLOC_WORKSPACE_MAX;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_DEVICES = 64;
std::mutex noalloc_mu;
void* noalloc_ptr[NOALLOC_DEVICES];   // device address of scratch on each device (null: not yet looked up)
bool noalloc_busy[NOALLOC_DEVICES];   // a live context holds that device's array

}  // namespace

extern "C" {

int kbe_workspace_query(const kbe_config* cfg, size_t* history_bytes, size_t* workspace_bytes,
                        size_t* obs_bytes) {
  Layout L;
  std::string why;
  int rc = make_layout(cfg, &L, &why);
  if (rc) return rc;
  if (history_bytes) *history_bytes = L.hist_bytes;
  if (workspace_bytes) *workspace_bytes = L.ws_bytes;
  if (obs_bytes) *obs_bytes = L.obs_bytes;
  return KBE_OK;
}


int kbe_create(const kbe_config* cfg, const double* hop, const kbe_pulse* pulse, void* d_history,
               size_t history_bytes, void* d_workspace, size_t workspace_bytes, void* d_obs, size_t obs_bytes,
               void* hip_stream, kbe_ctx** out) {
  return create_context(cfg, hop, pulse, d_history, history_bytes, d_workspace, workspace_bytes, d_obs, obs_bytes,
                        hip_stream, out, false);
}

int kbe_create_noalloc(const kbe_config* cfg, const double* hop, const kbe_pulse* pulse, void* d_history,
                       size_t history_bytes, void* d_obs, size_t obs_bytes, void* hip_stream, kbe_ctx** out) {
  if (!out) return KBE_ERR_INVALID_ARG;
  *out = nullptr;
  Layout L;
  std::string why;
  int rc = make_layout(cfg, &L, &why);
  if (rc) return rc;
  if (L.ws_bytes > NOALLOC_BYTES) return KBE_ERR_SHAPE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return KBE_ERR_HIP;
  if (dev < 0 || dev >= NOALLOC_DEVICES) return KBE_ERR_SHAPE;
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_ptr[dev]) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return KBE_ERR_HIP;
      noalloc_ptr[dev] = p;
    }
    if (noalloc_busy[dev]) return KBE_ERR_STATE;
    noalloc_busy[dev] = true;
    ws = noalloc_ptr[dev];
  }
  rc = create_context(cfg, hop, pulse, d_history, history_bytes, ws, NOALLOC_BYTES, d_obs, obs_bytes, hip_stream,
                      out, true);
  std::lock_guard<std::mutex> lock(noalloc_mu);
  if (rc) noalloc_busy[dev] = false;
  else (*out)->noalloc_dev = dev;
  return rc;
}

int kbe_step(kbe_ctx* ctx, int32_t nsteps) {
  if (!ctx || nsteps < 0) return KBE_ERR_INVALID_ARG;
  if (ctx->frozen) return ctx->fail(KBE_ERR_STATE, "the context's buffers were used by a reverse sweep");
  if ((int64_t)ctx->step + nsteps > ctx->cfg.nt_max) return ctx->fail(KBE_ERR_STATE, "step index would pass nt_max");
  for (int i = 0; i < nsteps; ++i) {
    int rc = ctx->one_step();
    if (rc) return rc;
  }
  return KBE_OK;
}

int32_t kbe_current_step(const kbe_ctx* ctx) { return ctx ? ctx->step : -1; }

int kbe_corrector_log(const kbe_ctx* ctx, int32_t first, int32_t count, int32_t* passes, double* changes) {
  if (!ctx || first < 0 || count < 0 || (int64_t)first + count > (int64_t)ctx->cfg.nt_max + 1) return KBE_ERR_INVALID_ARG;
  const int K = ctx->cfg.n_corr > 0 ? ctx->cfg.n_corr : 1;
  for (int i = 0; i < count; ++i) {
    int m = first + i;
    if (passes) passes[i] = ctx->passes[m];
    if (changes)
      for (int p = 0; p < ctx->cfg.n_corr; ++p) changes[(size_t)i * ctx->cfg.n_corr + p] = ctx->changes[(size_t)m * K + p];
  }
  return KBE_OK;
}

int kbe_observables(kbe_ctx* ctx, int32_t first, int32_t count, double* host_out) {
  if (!ctx || !host_out || first < 0 || count < 0 || (int64_t)first + count > (int64_t)ctx->cfg.nt_max + 1)
    return KBE_ERR_INVALID_ARG;
  int rc = ctx->check(hipStreamSynchronize(ctx->st), "stream synchronisation");
  if (rc) return rc;
  rc = ctx->check(hipMemcpy(host_out, ctx->obs + (size_t)first * KBE_NOBS, (size_t)count * KBE_NOBS * sizeof(double),
                            hipMemcpyDeviceToHost),
                  "observables copy");
  if (rc) return rc;
  for (int i = 0; i < count * KBE_NOBS; ++i)
    if (!std::isfinite(host_out[i])) return ctx->fail(KBE_ERR_NONFINITE, "non-finite observable");
  return KBE_OK;
}

void kbe_destroy(kbe_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->st);
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  if (ctx->noalloc_dev >= 0) {
    // the context's work has completed: the device's static workspace is free again
    std::lock_guard<std::mutex> lock(noalloc_mu);
    noalloc_busy[ctx->noalloc_dev] = false;
  }
  delete ctx;
}

const char* kbe_last_error(const kbe_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int kbe_buffer(const kbe_ctx* ctx, int32_t which, void** ptr, size_t* bytes) {
  if (!ctx || !ptr) return KBE_ERR_INVALID_ARG;
  int b;
  int c = ctx->cur;
  switch (which) {
    case KBE_BUF_SIGMA: b = B_SIGMA; break;
    case KBE_BUF_I_PREV: b = c == 0 ? B_IA : B_IB; break;
    case KBE_BUF_I_CUR: b = c == 0 ? B_IB : B_IA; break;
    case KBE_BUF_RHO_PREV: b = c == 0 ? B_RHOA : B_RHOB; break;
    case KBE_BUF_RHO_CUR: b = c == 0 ? B_RHOB : B_RHOA; break;
    case KBE_BUF_D_PREV: b = c == 0 ? B_DA : B_DB; break;
    case KBE_BUF_D_CUR: b = c == 0 ? B_DB : B_DA; break;
    case KBE_BUF_PROP: b = B_PROP; break;
    case KBE_BUF_COL0: b = B_COL0; break;
    case KBE_BUF_DIAG: b = B_DIAG; break;
    case KBE_BUF_ROWS: b = B_ROW64; break;
    default: return KBE_ERR_INVALID_ARG;
  }
  *ptr = ctx->ws + ctx->L.off[b];
  if (bytes) *bytes = ctx->L.bytes[b];
  return KBE_OK;
}

static int check_m(kbe_ctx* ctx, int32_t m, int lo) {
  if (!ctx) return KBE_ERR_INVALID_ARG;
  if (ctx->frozen) return ctx->fail(KBE_ERR_STATE, "the context's buffers were used by a reverse sweep");
  if (m < lo || m > ctx->cfg.nt_max) return ctx->fail(KBE_ERR_INVALID_ARG, "time-slice index out of range");
  return KBE_OK;
}

int kbe_stage_propagators(kbe_ctx* ctx, int32_t m, int32_t mode) {
  int rc = check_m(ctx, m, 1);
  if (rc) return rc;
  if (mode != 0 && mode != 1) return ctx->fail(KBE_ERR_INVALID_ARG, "mode must be 0 or 1");
  LaunchArgs a = ctx->args();
  return ctx->props(a, m, mode);
}

int kbe_stage_sigma(kbe_ctx* ctx, int32_t m) {
  int rc = check_m(ctx, m, 0);
  if (rc) return rc;
  LaunchArgs a = ctx->args();
  return ctx->check(kbe::launch_sigma(ctx->L.d, a, m, ctx->st), "self-energy launch");
}

int kbe_stage_sigma_direct(kbe_ctx* ctx, int32_t m) {
  int rc = check_m(ctx, m, 0);
  if (rc) return rc;
  const kbe_config& c = ctx->cfg;
  if (c.interaction != KBE_INT_INTERBAND || c.nky != 1 || c.nkx % 8 != 0)
    return ctx->fail(KBE_ERR_SHAPE, "the direct-sum self-energy needs the interband preset on a chain of 8j points");
  LaunchArgs a = ctx->args();
  return ctx->check(kbe::launch_sigma_direct(ctx->L.d, a, m, ctx->st), "direct self-energy launch");
}

int kbe_stage_collision(kbe_ctx* ctx, int32_t m) {
  int rc = check_m(ctx, m, 0);
  if (rc) return rc;
  LaunchArgs a = ctx->args();
  rc = ctx->check(kbe::launch_diag_I(ctx->L.d, a, m, ctx->st), "equal-time collision launch");
  if (!rc) rc = ctx->bulk_timed(a, m);
  if (!rc) rc = ctx->check(kbe::launch_row(ctx->L.d, a, m, KBE_ROW_EVAL, ctx->st), "collision-row launch");
  return rc;
}

int kbe_stage_update(kbe_ctx* ctx, int32_t m, int32_t mode) {
  int rc = check_m(ctx, m, 1);
  if (rc) return rc;
  if (mode != 0 && mode != 1) return ctx->fail(KBE_ERR_INVALID_ARG, "mode must be 0 or 1");
  LaunchArgs a = ctx->args();
  return ctx->check(kbe::launch_row(ctx->L.d, a, m, mode == 0 ? KBE_ROW_PREDICT : KBE_ROW_CORRECT, ctx->st),
                    "update launch");
}

int kbe_stage_observables(kbe_ctx* ctx, int32_t m) {
  int rc = check_m(ctx, m, 0);
  if (rc) return rc;
  return ctx->observe(m);
}

int kbe_stage_commit(kbe_ctx* ctx, int32_t m) {
  int rc = check_m(ctx, m, 1);
  if (rc) return rc;
  if (m != ctx->step + 1) return ctx->fail(KBE_ERR_STATE, "commit(m) must follow step m - 1");
  rc = ctx->dipole_kick(m);
  if (rc) return rc;
  ctx->cur ^= 1;
  ctx->step = m;
  return KBE_OK;
}

int kbe_rebuild_aux(kbe_ctx* ctx, int32_t m) {
  int rc = check_m(ctx, m, 0);
  if (rc) return rc;
  LaunchArgs a = ctx->args();
  return ctx->check(kbe::launch_aux(ctx->L.d, a, m, ctx->st), "aux launch");
}

int kbe_timing(kbe_ctx* ctx, int32_t enable) {
  if (!ctx) return KBE_ERR_INVALID_ARG;
  // events of an earlier window may still be pending on the stream: let them complete before
  // they are recorded again
  int rc = ctx->check(hipStreamSynchronize(ctx->st), "stream synchronisation");
  if (rc) return rc;
  ctx->timing = enable != 0;
  ctx->ev_used = 0;
  ctx->ev_m.clear();
  if (ctx->timing) {
    // two events per history-sum launch: at most n_corr + 1 passes per step, one more on the
    // dipole-kick slice, for every step up to nt_max
    size_t need = 2 * ((size_t)ctx->cfg.nt_max * (ctx->cfg.n_corr + 1) + 1);
    ctx->ev_m.reserve(need / 2);
    while (ctx->ev.size() < need) {
      hipEvent_t e;
      rc = ctx->check(hipEventCreate(&e), "hipEventCreate");
      if (rc) return rc;
      ctx->ev.push_back(e);
    }
  }
  return KBE_OK;
}

int kbe_timing_query(kbe_ctx* ctx, int64_t* launches, double* total_ms, double* algo_bytes) {
  if (!ctx) return KBE_ERR_INVALID_ARG;
  int rc = ctx->check(hipStreamSynchronize(ctx->st), "stream synchronisation");
  if (rc) return rc;
  double ms_sum = 0.0, bytes = 0.0;
  const Dims& d = ctx->L.d;
  for (size_t i = 0; i < ctx->ev_m.size(); ++i) {
    float ms = 0.f;
    rc = ctx->check(hipEventElapsedTime(&ms, ctx->ev[2 * i], ctx->ev[2 * i + 1]), "hipEventElapsedTime");
    if (rc) return rc;
    ms_sum += ms;
    double m = ctx->ev_m[i];
    bytes += 0.5 * m * (m + 1.0) * d.nk * d.C * (d.fp32 ? sizeof(float2) : sizeof(cplx));
  }
  if (launches) *launches = (int64_t)ctx->ev_m.size();
  if (total_ms) *total_ms = ms_sum;
  if (algo_bytes) *algo_bytes = bytes;
  return KBE_OK;
}

int kbe_adjoint_query(const kbe_config* cfg, size_t* adjoint_bytes) {
  if (!adjoint_bytes) return KBE_ERR_INVALID_ARG;
  Layout L;
  std::string why;
  int rc = make_layout(cfg, &L, &why);
  if (rc) return rc;
  if (cfg->precision != KBE_FP64 || cfg->n_corr != 1 || cfg->corr_tol != 0.0 || cfg->quad_points > 1 || cfg->nb > 2 ||
      cfg->interaction != KBE_INT_HUBBARD || cfg->nkx > 64)
    return KBE_ERR_SHAPE;
  *adjoint_bytes = adj_layout(L, nullptr);
  return KBE_OK;
}

int kbe_adjoint_attach(kbe_ctx* ctx, void* d_adjoint, size_t bytes) {
  if (!ctx || !d_adjoint) return KBE_ERR_INVALID_ARG;
  if (ctx->cfg.precision != KBE_FP64 || ctx->cfg.n_corr != 1 || ctx->cfg.corr_tol != 0.0 || ctx->L.d.qp > 1 ||
      ctx->L.d.nb > 2 || ctx->cfg.interaction != KBE_INT_HUBBARD || ctx->pulse.kind != KBE_PULSE_PEIERLS ||
      ctx->cfg.nkx > 64)
    return ctx->fail(KBE_ERR_SHAPE,
                     "the adjoint needs precision KBE_FP64, a fixed n_corr = 1 (corr_tol = 0), the trapezoid rule "
                     "(quad_points <= 1), nb <= 2, the Hubbard preset, the Peierls pulse and nkx <= 64");
  if (ctx->adj_obs >= 0) return ctx->fail(KBE_ERR_STATE, "a reverse sweep is in progress");
  size_t need = adj_layout(ctx->L, ctx->adj_off);
  if (bytes < need) return ctx->fail(KBE_ERR_INVALID_ARG, "adjoint workspace smaller than kbe_adjoint_query");
  ctx->adj = (char*)d_adjoint;
  return KBE_OK;
}

int kbe_adjoint_step(kbe_ctx* ctx, int32_t observable_id, double* grad_out, int32_t* steps_remaining) {
  if (!ctx) return KBE_ERR_INVALID_ARG;
  if (!ctx->adj) return ctx->fail(KBE_ERR_STATE, "no adjoint workspace attached");
  int nb = ctx->L.d.nb;
  bool norb = observable_id >= KBE_OBS_NORB && observable_id < KBE_OBS_NORB + nb;
  bool nband = observable_id >= KBE_OBS_NBAND && observable_id < KBE_OBS_NBAND + nb;
  if (!norb && !nband) return ctx->fail(KBE_ERR_INVALID_ARG, "observable must be an orbital or band occupation");
  int rc;
  if (ctx->adj_obs < 0) {
    if (ctx->step < 1) return ctx->fail(KBE_ERR_STATE, "no step to reverse");
    ctx->frozen = true;
    ctx->adj_obs = observable_id;
    ctx->adj_m = ctx->step;
    ctx->adj_cur = 0;
    rc = ctx->adj_seed(observable_id);
    if (rc) return rc;
  } else if (observable_id != ctx->adj_obs) {
    return ctx->fail(KBE_ERR_STATE, "observable differs from the one the sweep was seeded with");
  }
  if (ctx->adj_m < 1) return ctx->fail(KBE_ERR_STATE, "no step left to reverse");
  rc = ctx->adj_reverse(ctx->adj_m);
  if (rc) return rc;
  ctx->adj_m -= 1;
  if (steps_remaining) *steps_remaining = ctx->adj_m;
  if (grad_out) {
    rc = ctx->check(hipMemcpyAsync(grad_out, ctx->abuf<double>(A_THETA), 3 * sizeof(double), hipMemcpyDeviceToHost,
                                   ctx->st),
                    "gradient copy");
    if (!rc) rc = ctx->check(hipStreamSynchronize(ctx->st), "stream synchronisation");
    if (rc) return rc;
    for (int i = 0; i < 3; ++i)
      if (!std::isfinite(grad_out[i])) return ctx->fail(KBE_ERR_NONFINITE, "non-finite gradient");
  }
  return KBE_OK;
}

}  // extern "C"
