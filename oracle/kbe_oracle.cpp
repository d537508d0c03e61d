// TEST INFRASTRUCTURE -- NOT PART OF THE PRODUCT PATH.
//
// Plain, slow, FP64 CPU reference of the Kadanoff-Baym propagation step of
// arXiv 2505.19467 ("GPU Acceleration of Non-equilibrium Green's Function
// Calculation using OpenACC and CUDA FORTRAN"). Only the tests, the smoke check
// and the CPU-baseline leg of the benchmark load this library. It shares no code,
// header or table with the HIP library, and it never calls it.
//
// Every function follows a passage of the paper (cited by section / equation /
// algorithm) or, where the paper is silent, the reading listed in the design
// notes (the same reading is restated at each function):
//
//   k grid ............ eq. (kj): k_j = -pi + 2 pi j / n per axis (0-based j)
//   Hamiltonian ....... Sec. "Computational Kernels", eq. (Htotal)/(ham), with a
//                       Peierls substitution k -> k - A(t) pol for the pulse
//   self-energy ....... eq. (2BSE) (second Born), evaluated in real space
//   collision integral  eq. (CI) in its Langreth "left" form, trapezoid rule (the
//                       second-order quadrature the paper states), or Gregory end
//                       corrections with more points per end (quad_points > 1)
//   propagation ....... Algorithm "prop" (predictor, corrector passes -- a fixed
//                       number, or up to that number until the row changes by at
//                       most a tolerance -- and re-evaluation after the step) with an
//                       exponential-midpoint solve of eq. (Green)
//   dipole pulse ...... eq. (dipole): E(t) = I delta(t - t0), d_k = 1, coupling bands 0 (v)
//                       and 1 (c), integrated across the delta as the kick exp(-i I sigma_x)
//                       applied to the completed slice nearest t0
//
// Conventions: G^<(t,t') = i<c^dag(t') c(t)>, G^>(t,t') = -i<c(t) c^dag(t')>;
// G^{<,>}(t',t) = -[G^{<,>}(t,t')]^dag; rho(t) = -i G^<(t,t).
//
// Storage (oracle-private): row j of the two-time lower triangle is an array
// [t'=0..j][k][comp(0:<,1:>)][a][b] of complex numbers.
//
// Every routine is written once for a generic real type R. R = double is the oracle;
// R = Dual<3> (value + three directional derivatives, forward-mode automatic
// differentiation) gives the tangent-linear model: the exact derivatives of the same
// computation with respect to the pulse amplitude, the pulse frequency and U.
//
// Pins (tests/test_oracle_pins.py, CPU only):
//   sigma_row ....... eq. (2BSE) direct double momentum sums (interband preset, with the
//                     paper's allind_kpk index map) and the Hubbard momentum convolution;
//                     conserving pairing (sum_k tr[S^> G^< - S^< G^>] imaginary)
//   collision_row ... exact on piecewise-linear integrands (trapezoid), zero at t = 0
//   quadrature ...... Gregory weights: the classical 3- and 4-point values, exactness on
//                     polynomials of the expected degree for every interval length, exact
//                     collision rows on polynomial histories
//   propagators ..... scipy expm of -i h dt and of the augmented phi_1 matrix
//   eigh, initial ... numpy eigh; Fermi-Dirac density; mu = 0 by particle-hole symmetry
//   dipole kick ..... U = 0 closed form with the kick (the order of the kick and the band
//                     propagation, its phase and its slice), exact N conservation; second-order
//                     convergence across the kick with a density-dependent mean field
//   interband HF .... one electron in a pure state: no self-interaction, so TDHF converges at
//                     second order to the exact one-electron evolution under h0 - U P_c
//   time stepping ... U = 0 closed form, exact N conservation, energy balance O(dt^2),
//                     dt-convergence ratio 4, TDHF limit vs RK4
//   symmetry ........ full-square mode: the upper triangle propagated on its own with the
//                     t'-equation and right-form collision integrals equals -G^dag of the
//                     lower one to rounding (Hubbard and interband presets); rho Hermitian
//   tangent-linear .. R = double run reproduced bit-for-bit by the value part; derivatives
//                     against central finite differences of the double oracle
//   corrector tol ... tolerance 0 reproduces the fixed-count run bit for bit, an infinite one
//                     the single-pass run; the changes shrink geometrically pass by pass and
//                     the stopping pass is the first whose change is at most the tolerance

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include <omp.h>

namespace {

// ---------------------------------------------------------------- real types
// Forward-mode dual number: value and N directional derivatives.
template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0.0) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
  Dual(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
};
template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r;
}
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r;
}
template <int N> inline Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r;
}
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r;
}
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
template <int N> inline Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> inline Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> inline Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, double b) {
  Dual<N> r; r.v = a.v * b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b; return r;
}
template <int N> inline Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N> inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> inline Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { a = a + b; return a; }
template <int N> inline Dual<N>& operator-=(Dual<N>& a, const Dual<N>& b) { a = a - b; return a; }
template <int N> inline Dual<N> chain(const Dual<N>& a, double f, double df) {
  Dual<N> r; r.v = f; for (int i = 0; i < N; ++i) r.d[i] = df * a.d[i]; return r;
}
template <int N> inline Dual<N> sqrt(const Dual<N>& a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
template <int N> inline Dual<N> exp(const Dual<N>& a) { double e = std::exp(a.v); return chain(a, e, e); }
template <int N> inline Dual<N> sin(const Dual<N>& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
template <int N> inline Dual<N> cos(const Dual<N>& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
template <int N> inline Dual<N> fabs(const Dual<N>& a) { return a.v < 0 ? -a : a; }
using std::cos;
using std::exp;
using std::fabs;
using std::sin;
using std::sqrt;
inline double val(double x) { return x; }
template <int N> inline double val(const Dual<N>& x) { return x.v; }

typedef Dual<3> D3;

template <class R>
struct Cx {
  R re, im;
  Cx() : re(0.0), im(0.0) {}
  Cx(R r) : re(r), im(0.0) {}
  Cx(R r, R i) : re(r), im(i) {}
};
template <class R> inline Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R> inline Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R> inline Cx<R> operator-(Cx<R> a) { return {-a.re, -a.im}; }
template <class R> inline Cx<R> operator*(Cx<R> a, Cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R> inline Cx<R> operator*(Cx<R> a, double s) { return {a.re * s, a.im * s}; }
template <class R> inline Cx<R> scale(Cx<R> a, R s) { return {a.re * s, a.im * s}; }
template <class R> inline Cx<R> conj(Cx<R> a) { return {a.re, -a.im}; }
template <class R> inline Cx<R>& operator+=(Cx<R>& a, Cx<R> b) { a.re += b.re; a.im += b.im; return a; }
template <class R> inline Cx<R>& operator-=(Cx<R>& a, Cx<R> b) { a.re -= b.re; a.im -= b.im; return a; }
template <class R> inline Cx<R> cexpi(R x) { using std::cos; using std::sin; return {cos(x), sin(x)}; }
template <class R> inline R abs2(Cx<R> a) { return a.re * a.re + a.im * a.im; }
template <class R> inline Cx<R> imag_unit() { return Cx<R>(R(0.0), R(1.0)); }

// ---------------------------------------------------------------- parameters
// Mirrors OracleParams in oracle/oracle.py (ctypes); plain data.
struct Params {
  int32_t nkx, nky, nb, spin_deg, interaction, hf, corr, n_corr, nt, quad_points, pulse_kind;
  double dt, U, temp, filling, amp, omega, t0, width, polx, poly;
  double corr_tol;  // > 0: corrector passes stop once the row changes by at most this
};
enum { INT_HUBBARD = 0, INT_INTERBAND = 1 };
enum { PULSE_PEIERLS = 0, PULSE_DIPOLE_KICK = 1 };
enum {
  OBS_T = 0, OBS_N, OBS_EKIN, OBS_EHF, OBS_ECORR, OBS_ETOT, OBS_JX, OBS_JY, OBS_A,
  OBS_NORB = 9, OBS_NBAND = 13, NOBS = 17
};

// The three parameters a gradient is taken with respect to, in the run's real type.
template <class R>
struct Theta {
  R amp, omega, U;
};

struct Grid {
  int nkx, nky, nk, nb, dim;
  std::vector<double> kx, ky;  // eq. (kj)
  explicit Grid(const Params& p) : nkx(p.nkx), nky(p.nky), nk(p.nkx * p.nky), nb(p.nb) {
    dim = (p.nky == 1) ? 1 : 2;
    kx.resize(nkx);
    ky.resize(nky);
    for (int j = 0; j < nkx; ++j) kx[j] = -M_PI + 2.0 * M_PI * j / nkx;
    for (int j = 0; j < nky; ++j) ky[j] = -M_PI + 2.0 * M_PI * j / nky;
  }
  // flattened k index: k = ix * nky + iy
  int ix(int k) const { return k / nky; }
  int iy(int k) const { return k % nky; }
};

// ---------------------------------------------------------------- small dense matrices
// n x n complex matrices in row-major arrays.
template <class R>
void mm(int n, const Cx<R>* A, const Cx<R>* B, Cx<R>* out) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      Cx<R> s;
      for (int l = 0; l < n; ++l) s += A[i * n + l] * B[l * n + j];
      out[i * n + j] = s;
    }
}
template <class R>
void adjoint(int n, const Cx<R>* A, Cx<R>* out) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[j * n + i] = conj(A[i * n + j]);
}

// Eigen-decomposition of a Hermitian matrix by cyclic complex Jacobi rotations.
// On exit w holds the eigenvalues in ascending order and the columns of Vec the
// eigenvectors (A = Vec diag(w) Vec^dag).
template <class R>
void eigh(int n, const Cx<R>* Ain, R* w, Cx<R>* Vec) {
  typedef Cx<R> C;
  std::vector<C> A(Ain, Ain + n * n);
  for (int i = 0; i < n * n; ++i) Vec[i] = C();
  for (int i = 0; i < n; ++i) Vec[i * n + i] = C(1.0);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) (p == q ? dia : off) += val(abs2(A[p * n + q]));
    if (off <= 1e-34 * (dia + 1e-300)) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        C apq = A[p * n + q];
        if (std::sqrt(val(abs2(apq))) < 1e-300) continue;
        R r = sqrt(abs2(apq));
        C ph = scale(apq, R(1.0) / r);  // e^{i phi}
        R a = A[p * n + p].re, b = A[q * n + q].re;
        // rotate the real symmetric problem [[a, r], [r, b]]
        R theta = (b - a) / (2.0 * r);
        R t = (val(theta) >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        R c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        // W = diag(1, e^{-i phi}) * [[c, s], [-s, c]] on the (p, q) plane
        C wpp(c), wpq(s), wqp = scale(conj(ph), -s), wqq = scale(conj(ph), c);
        for (int i = 0; i < n; ++i) {  // A <- A W
          C aip = A[i * n + p], aiq = A[i * n + q];
          A[i * n + p] = aip * wpp + aiq * wqp;
          A[i * n + q] = aip * wpq + aiq * wqq;
        }
        for (int j = 0; j < n; ++j) {  // A <- W^dag A
          C apj = A[p * n + j], aqj = A[q * n + j];
          A[p * n + j] = conj(wpp) * apj + conj(wqp) * aqj;
          A[q * n + j] = conj(wpq) * apj + conj(wqq) * aqj;
        }
        A[p * n + q] = C();
        A[q * n + p] = C();
        A[p * n + p].im = 0.0;
        A[q * n + q].im = 0.0;
        for (int i = 0; i < n; ++i) {  // Vec <- Vec W
          C vip = Vec[i * n + p], viq = Vec[i * n + q];
          Vec[i * n + p] = vip * wpp + viq * wqp;
          Vec[i * n + q] = vip * wpq + viq * wqq;
        }
      }
  }
  // sort ascending
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::vector<R> d(n);
  for (int i = 0; i < n; ++i) d[i] = A[i * n + i].re;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return val(d[x]) < val(d[y]); });
  std::vector<C> V2(n * n);
  for (int c = 0; c < n; ++c) {
    w[c] = d[idx[c]];
    for (int i = 0; i < n; ++i) V2[i * n + c] = Vec[i * n + idx[c]];
  }
  std::copy(V2.begin(), V2.end(), Vec);
}

// f(h) = U diag(f(w)) U^dag for a Hermitian h.
template <class R, class F>
void matfun(int n, const Cx<R>* h, F f, Cx<R>* out) {
  std::vector<R> w(n);
  std::vector<Cx<R>> U(n * n);
  eigh(n, h, w.data(), U.data());
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      Cx<R> s;
      for (int b = 0; b < n; ++b) s += U[i * n + b] * f(w[b]) * conj(U[j * n + b]);
      out[i * n + j] = s;
    }
}

// ---------------------------------------------------------------- model
// Pulse A(t) = amp sin(omega t) exp(-((t - t0)/width)^2), along pol (the dipole pulse has
// no vector potential).
template <class R>
R pulse_A(const Params& p, const Theta<R>& th, double t) {
  if (p.pulse_kind == PULSE_DIPOLE_KICK) return R(0.0);
  double x = (t - p.t0) / p.width;
  return th.amp * sin(th.omega * t) * std::exp(-x * x);
}

// h0(k - A pol) = T0 + sum_d [T_d e^{i q_d} + T_d^dag e^{-i q_d}], q = k - A pol.
template <class R>
void h0(const Params& p, const Grid& g, const Cx<R>* hop, int k, R A, Cx<R>* out) {
  typedef Cx<R> C;
  int nb = g.nb;
  R q[2] = {g.kx[g.ix(k)] - A * p.polx, g.ky[g.iy(k)] - A * p.poly};
  for (int a = 0; a < nb; ++a)
    for (int b = 0; b < nb; ++b) {
      C s = hop[a * nb + b];
      for (int d = 0; d < g.dim; ++d) {
        const C* T = hop + (1 + d) * nb * nb;
        s += T[a * nb + b] * cexpi(q[d]) + conj(T[b * nb + a]) * cexpi(-q[d]);
      }
      out[a * nb + b] = s;
    }
}

// velocity d h0 / d k_d at k - A pol: i (T_d e^{i q_d} - T_d^dag e^{-i q_d})
template <class R>
void vel(const Params& p, const Grid& g, const Cx<R>* hop, int k, R A, int d, Cx<R>* out) {
  typedef Cx<R> C;
  int nb = g.nb;
  R q[2] = {g.kx[g.ix(k)] - A * p.polx, g.ky[g.iy(k)] - A * p.poly};
  for (int a = 0; a < nb; ++a)
    for (int b = 0; b < nb; ++b) {
      if (d >= g.dim) { out[a * nb + b] = C(); continue; }
      const C* T = hop + (1 + d) * nb * nb;
      out[a * nb + b] = imag_unit<R>() * (T[a * nb + b] * cexpi(q[d]) - conj(T[b * nb + a]) * cexpi(-q[d]));
    }
}

// Mean-field (first-order) self-energy from the local density matrix
// rho_loc = N_k^{-1} sum_k rho(k).
//  Hubbard (intra-orbital U, opposite spins): Sigma_ab = delta_ab U rho_loc,aa.
//  Interband, eq. (ham): Hartree U n_c on v and U n_v on c, Fock -U rho_loc,vc on
//  the off-diagonal.
template <class R>
void hf_field(const Params& p, const Theta<R>& th, const Grid& g, const std::vector<Cx<R>>& rho, Cx<R>* out) {
  typedef Cx<R> C;
  int nb = g.nb, nbb = nb * nb;
  std::vector<C> loc(nbb);
  for (int k = 0; k < g.nk; ++k)
    for (int i = 0; i < nbb; ++i) loc[i] += rho[k * nbb + i];
  for (int i = 0; i < nbb; ++i) loc[i] = loc[i] * (1.0 / g.nk);
  for (int i = 0; i < nbb; ++i) out[i] = C();
  if (!p.hf) return;
  if (p.interaction == INT_HUBBARD) {
    for (int a = 0; a < nb; ++a) out[a * nb + a] = C(th.U * loc[a * nb + a].re);
  } else {
    out[0] = C(th.U * loc[3].re);
    out[3] = C(th.U * loc[0].re);
    out[1] = scale(loc[1], -th.U);
    out[2] = scale(loc[2], -th.U);
  }
}

// The dipole pulse of eq. (dipole), E(t) = I delta(t - t0) with d_k = 1: H_ext(t) = E(t) X,
// X the matrix with ones between band 0 (v) and band 1 (c). Across the delta the equation of
// motion reduces to i dG/dt = E(t) X G, so G(t0+, t') = exp(-i I X) G(t0-, t') with
// exp(-i I X) = cos(I) 1 - i sin(I) X. On the time grid the kick sits at the grid time t_{m0}
// nearest t0 (m0 = floor(t0 / dt + 1/2)): once slice m0 is complete (its observables are the
// values just before the kick), it is replaced by the kicked slice and its self-energy and
// collision integrals are evaluated again on it (dipole_kick below).
inline int kick_slice(const Params& p) { return (int)std::floor(p.t0 / p.dt + 0.5); }
template <class R>
void kick_matrix(const Theta<R>& th, Cx<R>* K) {
  using std::cos;
  using std::sin;
  R c = cos(th.amp), s = sin(th.amp);
  K[0] = Cx<R>(c);
  K[3] = Cx<R>(c);
  K[1] = Cx<R>(R(0.0), -s);
  K[2] = Cx<R>(R(0.0), -s);
}

// k-independent one-body term: the -U c_c^dag c_c term of eq. (ham) (interband only).
template <class R>
void onebody_extra(const Params& p, const Theta<R>& th, int nb, Cx<R>* out) {
  for (int i = 0; i < nb * nb; ++i) out[i] = Cx<R>();
  if (p.interaction == INT_INTERBAND) out[3] = Cx<R>(-th.U);
}

// ---------------------------------------------------------------- state
template <class R>
struct State {
  typedef Cx<R> C;
  const Params& p;
  Theta<R> th;
  Grid g;
  std::vector<C> hop;
  int nbb, blk;                    // nb^2, 2 nb^2 (one (t,t') block: lesser then greater)
  std::vector<std::vector<C>> rows;  // rows[j]: [t'][k][comp][a][b]
  std::vector<C> rho_prev, rho_cur, D_prev, D_cur;  // [k][a][b]
  std::vector<C> I_prev, I_cur;    // [t'][k][comp][a][b], t' = 0..m
  std::vector<C> sig;              // [j][k][comp][a][b], j = 0..m
  std::vector<int> passes;         // corrector passes taken at each step (index m)
  std::vector<double> changes;     // after each pass: max |G_new - G_old| over row m
  std::vector<int> unconverged;    // 1 at step m if all n_corr passes ended above corr_tol
  State(const Params& pp, const Theta<R>& t, const double* hopd) : p(pp), th(t), g(pp) {
    nbb = g.nb * g.nb;
    blk = 2 * nbb;
    hop.resize(3 * nbb);
    for (int i = 0; i < 3 * nbb; ++i) hop[i] = C(hopd[2 * i], hopd[2 * i + 1]);
  }
  C* at(int j, int tp, int k) { return rows[j].data() + ((size_t)tp * g.nk + k) * blk; }
};

// Equal-time block of G from rho: G^< = i rho, G^> = -i (1 - rho).
template <class R>
void set_diag_block(int nb, const Cx<R>* rho, Cx<R>* blk) {
  typedef Cx<R> C;
  const C I1 = imag_unit<R>();
  for (int a = 0; a < nb; ++a)
    for (int b = 0; b < nb; ++b) {
      C r = rho[a * nb + b];
      blk[a * nb + b] = I1 * r;
      C one_minus = (a == b ? C(1.0) : C()) - r;
      blk[nb * nb + a * nb + b] = -(I1 * one_minus);
    }
}

// Initial state: uncorrelated Fermi-Dirac density of h0(k - A(0)) at temperature T,
// chemical potential by bisection so that N_k^{-1} sum_k tr rho = nb * filling.
// (The paper starts from a given G; the configurations ask for an uncorrelated
// state at half filling and temperature T.) Computed in double: it does not depend on
// the pulse (A(0) = 0 for the sin pulse) nor on U.
double initial_state(const Params& p, const Grid& g, const Cx<double>* hop, std::vector<Cx<double>>& rho) {
  typedef Cx<double> C;
  int nb = g.nb, nbb = nb * nb;
  std::vector<double> w(g.nk * nb);
  std::vector<C> U(g.nk * nbb), h(nbb);
  Theta<double> th{p.amp, p.omega, p.U};
  double A0 = pulse_A(p, th, 0.0);
  for (int k = 0; k < g.nk; ++k) {
    h0(p, g, hop, k, A0, h.data());
    eigh(nb, h.data(), &w[k * nb], &U[k * nbb]);
  }
  auto fermi = [&](double e, double mu) { return 1.0 / (1.0 + std::exp((e - mu) / p.temp)); };
  double lo = *std::min_element(w.begin(), w.end()) - 50.0 * p.temp - 1.0;
  double hi = *std::max_element(w.begin(), w.end()) + 50.0 * p.temp + 1.0;
  double target = nb * p.filling * g.nk;
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    double n = 0.0;
    for (double e : w) n += fermi(e, mid);
    if (n < target) lo = mid; else hi = mid;
    if (hi - lo < 1e-15 * std::max(1.0, std::fabs(mid))) break;
  }
  double mu = 0.5 * (lo + hi);
  rho.assign(g.nk * nbb, C());
  for (int k = 0; k < g.nk; ++k)
    for (int a = 0; a < nb; ++a)
      for (int b = 0; b < nb; ++b) {
        C s;
        for (int c = 0; c < nb; ++c)
          s += U[k * nbb + a * nb + c] * fermi(w[k * nb + c], mu) * conj(U[k * nbb + b * nb + c]);
        rho[k * nbb + a * nb + b] = s;
      }
  return mu;
}

// ---------------------------------------------------------------- self-energy
// Real-space transforms over the k grid of eq. (kj):
//   g(R) = N_k^{-1} sum_k e^{i k.R} G(k),     Sigma(k) = sum_R e^{-i k.R} Sigma(R).
// Written as two 1D direct sums (the exponential factorises over the axes).
template <class R>
struct Dft {
  typedef Cx<R> C;
  int nx, ny;
  std::vector<C> ex, ey;  // ex[j * nx + R] = e^{i kx_j R}
  explicit Dft(const Grid& g) : nx(g.nkx), ny(g.nky) {
    ex.resize(nx * nx);
    ey.resize(ny * ny);
    for (int j = 0; j < nx; ++j)
      for (int r = 0; r < nx; ++r) ex[j * nx + r] = C(std::cos(g.kx[j] * r), std::sin(g.kx[j] * r));
    for (int j = 0; j < ny; ++j)
      for (int r = 0; r < ny; ++r) ey[j * ny + r] = C(std::cos(g.ky[j] * r), std::sin(g.ky[j] * r));
  }
  // g(s R) = N_k^{-1} sum_k e^{i s k.R} G(k) for R = (rx, ry), rx in [0, nx), ry in [0, ny)
  // and s = +1 or -1 (the lattice vector R or -R); in indexed k = ix*ny + iy, out R = rx*ny + ry.
  void to_real(const C* in, C* out, int s = +1) const {
    std::vector<C> tmp(nx * ny);
    for (int ix = 0; ix < nx; ++ix)
      for (int ry = 0; ry < ny; ++ry) {
        C acc;
        for (int iy = 0; iy < ny; ++iy) {
          C e = ey[iy * ny + ry];
          acc += in[ix * ny + iy] * (s > 0 ? e : conj(e));
        }
        tmp[ix * ny + ry] = acc;
      }
    for (int rx = 0; rx < nx; ++rx)
      for (int ry = 0; ry < ny; ++ry) {
        C acc;
        for (int ix = 0; ix < nx; ++ix) {
          C e = ex[ix * nx + rx];
          acc += tmp[ix * ny + ry] * (s > 0 ? e : conj(e));
        }
        out[rx * ny + ry] = acc * (1.0 / (nx * ny));
      }
  }
  // S(k) = sum_R e^{-i k.R} S(R).
  void to_k(const C* in, C* out) const {
    std::vector<C> tmp(nx * ny);
    for (int rx = 0; rx < nx; ++rx)
      for (int iy = 0; iy < ny; ++iy) {
        C s;
        for (int ry = 0; ry < ny; ++ry) s += in[rx * ny + ry] * conj(ey[iy * ny + ry]);
        tmp[rx * ny + iy] = s;
      }
    for (int ix = 0; ix < nx; ++ix)
      for (int iy = 0; iy < ny; ++iy) {
        C s;
        for (int rx = 0; rx < nx; ++rx) s += tmp[rx * ny + iy] * conj(ex[ix * nx + rx]);
        out[ix * ny + iy] = s;
      }
  }
};

// Second-Born self-energy, eq. (2BSE), for pairs of times: out[j] = Sigma(k; t_x, t_j) from the
// forward line fwd[j] = G(k; t_x, t_j) and the backward line bwd[j] = G(k; t_j, t_x), j = 0..m.
// In real space the double k-sum of eq. (2BSE) becomes a product at each lattice vector R
// (momentum conservation): for the Hubbard preset (opposite-spin bubble)
//   Sigma^<_ab(R; t,t') = U^2 G^<_ab(R; t,t') G^<_ab(R; t,t') G^>_ba(-R; t',t)
// and for the paper's interband preset (jbar = other band)
//   Sigma^<_jm(R) = U^2 G^>_{mbar jbar}(-R; t',t) [G^<_{jbar mbar}(R) G^<_jm(R)
//                                                - G^<_{j mbar}(R) G^<_{jbar m}(R)],
// with lesser and greater swapped for Sigma^>. U(t) is constant here.
// fwd, bwd, out: [j][k][comp][a][b].
template <class R>
void sigma_pairs(const Params& p, const Theta<R>& th, const Grid& g, int m, const Cx<R>* fwd, const Cx<R>* bwd,
                 Cx<R>* out) {
  typedef Cx<R> C;
  int nb = g.nb, nbb = nb * nb, blk = 2 * nbb, nk = g.nk;
  Dft<R> dft(g);
  R UU = th.U * th.U;
  if (!p.corr) {
    std::fill(out, out + (size_t)(m + 1) * nk * blk, C());
    return;
  }
#pragma omp parallel for schedule(dynamic)
  for (int j = 0; j <= m; ++j) {
    // gf[comp][a][b][R] = G^comp_ab(R; t_x, t_j); gb[comp][a][b][R] = G^comp_ab(-R; t_j, t_x)
    std::vector<C> gf(blk * nk), gb(blk * nk), in(nk), o(nk), sr(blk * nk);
    for (int comp = 0; comp < 2; ++comp)
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) {
          for (int k = 0; k < nk; ++k) in[k] = fwd[((size_t)j * nk + k) * blk + comp * nbb + a * nb + b];
          dft.to_real(in.data(), &gf[((comp * nb + a) * nb + b) * nk]);
          for (int k = 0; k < nk; ++k) in[k] = bwd[((size_t)j * nk + k) * blk + comp * nbb + a * nb + b];
          dft.to_real(in.data(), &gb[((comp * nb + a) * nb + b) * nk], -1);
        }
    auto G = [&](const std::vector<C>& v, int comp, int a, int b, int Rv) -> C {
      return v[((comp * nb + a) * nb + b) * nk + Rv];
    };
    for (int comp = 0; comp < 2; ++comp) {
      int oth = 1 - comp;  // Sigma^< uses G^> on the backward line, and vice versa
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b)
          for (int Rv = 0; Rv < nk; ++Rv) {
            C s;
            if (p.interaction == INT_HUBBARD) {
              s = G(gf, comp, a, b, Rv) * G(gf, comp, a, b, Rv) * G(gb, oth, b, a, Rv);
            } else {
              int ab = 1 - a, bb = 1 - b;
              C back = G(gb, oth, bb, ab, Rv);
              s = back * (G(gf, comp, ab, bb, Rv) * G(gf, comp, a, b, Rv) -
                          G(gf, comp, a, bb, Rv) * G(gf, comp, ab, b, Rv));
            }
            sr[((comp * nb + a) * nb + b) * nk + Rv] = scale(s, UU);
          }
    }
    for (int comp = 0; comp < 2; ++comp)
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) {
          dft.to_k(&sr[((comp * nb + a) * nb + b) * nk], o.data());
          for (int k = 0; k < nk; ++k) out[((size_t)j * nk + k) * blk + comp * nbb + a * nb + b] = o[k];
        }
  }
}

// Self-energy on row m: Sigma(k; t_m, t_j), j = 0..m, from row m alone, the backward line
// being G(k; t_j, t_m) = -[G(k; t_m, t_j)]^dag. row, out: [j][k][comp][a][b].
template <class R>
void sigma_row(const Params& p, const Theta<R>& th, const Grid& g, int m, const Cx<R>* row, Cx<R>* out) {
  typedef Cx<R> C;
  int nb = g.nb, nbb = nb * nb, blk = 2 * nbb, nk = g.nk;
  std::vector<C> bwd((size_t)(m + 1) * nk * blk);
  for (size_t jk = 0; jk < (size_t)(m + 1) * nk; ++jk)
    for (int comp = 0; comp < 2; ++comp)
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b)
          bwd[jk * blk + comp * nbb + a * nb + b] = -conj(row[jk * blk + comp * nbb + b * nb + a]);
  sigma_pairs(p, th, g, m, row, bwd.data(), out);
}

// ---------------------------------------------------------------- collision integral
// Quadrature weights of eq. (CI). The paper states a second-order rule, taken here as the
// trapezoid; with quad_points = q > 1 the end weights carry Gregory corrections.
// The trapezoid sum of a polynomial f on the nodes 0..N differs from its integral only by
// end terms (Euler-Maclaurin): sum_j f(j) - int_0^N f = (f(0) + f(N))/2
//   + sum_{k>=1} B_{2k}/(2k)! [f^{(2k-1)}(N) - f^{(2k-1)}(0)].
// Corrections c_0..c_{q-1} on the first q nodes cancel the left end's terms for every
// f of degree < q:  sum_{j<q} c_j j^d = -1/2 [d = 0] + [d odd] B_{d+1} / (d+1),  d = 0..q-1,
// and the mirrored ones the right end's. On [0, N] node j gets
//   w_j = 1 + c_j [j < q'] + c_{N-j} [N - j < q'],  q' = min(q, N + 1),
// so short intervals use fewer points (q' = N + 1 gives the closed Newton-Cotes rule on all
// nodes, q' = 1 the trapezoid, N = 0 the empty integral). q = 1 is the trapezoid rule.
const int QUAD_MAX = 8;

// Bernoulli numbers B_0..B_n from their recurrence sum_{k<=n} C(n+1, k) B_k = 0 (B_0 = 1).
std::vector<double> bernoulli(int n) {
  std::vector<double> B(n + 1, 0.0);
  B[0] = 1.0;
  for (int i = 1; i <= n; ++i) {
    double s = 0.0, binom = 1.0;  // C(i + 1, k)
    for (int k = 0; k < i; ++k) {
      s += binom * B[k];
      binom = binom * (i + 1 - k) / (k + 1);
    }
    B[i] = -s / (i + 1);
  }
  return B;
}

// c[q][j], q = 1..QUAD_MAX: the end corrections above, by Gaussian elimination with partial
// pivoting on the q x q system.
const std::vector<std::vector<double>>& gregory_corrections() {
  static const std::vector<std::vector<double>> table = [] {
    std::vector<std::vector<double>> c(QUAD_MAX + 1);
    std::vector<double> B = bernoulli(QUAD_MAX + 1);
    for (int q = 1; q <= QUAD_MAX; ++q) {
      std::vector<double> A(q * q), b(q);
      for (int d = 0; d < q; ++d) {
        for (int j = 0; j < q; ++j) A[d * q + j] = std::pow((double)j, d);  // 0^0 = 1
        b[d] = (d == 0 ? -0.5 : 0.0) + (d % 2 == 1 ? B[d + 1] / (d + 1) : 0.0);
      }
      for (int col = 0; col < q; ++col) {
        int piv = col;
        for (int r = col + 1; r < q; ++r)
          if (std::fabs(A[r * q + col]) > std::fabs(A[piv * q + col])) piv = r;
        for (int j = 0; j < q; ++j) std::swap(A[col * q + j], A[piv * q + j]);
        std::swap(b[col], b[piv]);
        for (int r = col + 1; r < q; ++r) {
          double f = A[r * q + col] / A[col * q + col];
          for (int j = col; j < q; ++j) A[r * q + j] -= f * A[col * q + j];
          b[r] -= f * b[col];
        }
      }
      c[q].assign(q, 0.0);
      for (int r = q - 1; r >= 0; --r) {
        double s = b[r];
        for (int j = r + 1; j < q; ++j) s -= A[r * q + j] * c[q][j];
        c[q][r] = s / A[r * q + r];
      }
    }
    return c;
  }();
  return table;
}

// Weight of node j on [0, N] (N = 0: the empty integral).
double quad_weight(const Params& p, int j, int N) {
  if (N <= 0) return 0.0;
  int q = std::min<int>(std::max<int>(p.quad_points, 1), N + 1);
  const std::vector<double>& c = gregory_corrections()[q];
  double w = 1.0;
  if (j < q) w += c[j];
  if (N - j < q) w += c[N - j];
  return w;
}

// Collision integrals of row m, eq. (CI), in the Langreth left form (reading of the
// paper's right-form expression that needs no self-energy history):
//   I^{<,>}(t_m, t') = int_0^{t_m} dtb Sigma^R(t_m, tb) G^{<,>}(tb, t')
//                    + int_0^{t'}  dtb Sigma^{<,>}(t_m, tb) G^A(tb, t'),
//   Sigma^R = Sigma^> - Sigma^< (tb < t_m),  G^A(tb,t') = -(G^> - G^<)(tb, t') (tb < t'),
// on the grid with the weights of quad_weight (trapezoid by default), for t' = t_0 .. t_m.
// hist(j, t', k) returns the stored block (j >= t'); blocks above the diagonal come from
// G(j, t') = -[G(t', j)]^dag, unless full_square, when hist returns G(t_j, t') for any pair.
template <class R, class Hist>
void collision_row(const Params& p, const Grid& g, int m, Hist hist, const Cx<R>* sig, Cx<R>* Iout,
                   bool full_square = false) {
  typedef Cx<R> C;
  int nb = g.nb, nbb = nb * nb, blk = 2 * nbb, nk = g.nk;
  double dt = p.dt;
#pragma omp parallel for schedule(dynamic)
  for (int k = 0; k < nk; ++k) {
    std::vector<C> Gb(blk), SR(nbb), GR(nbb), tmp(nbb), acc(blk);
    for (int tp = 0; tp <= m; ++tp) {
      std::fill(acc.begin(), acc.end(), C());
      for (int j = 0; j <= m; ++j) {
        // G(t_j, t')
        if (j >= tp || full_square) {  // full_square: hist holds G(t_j, t') for every pair
          const C* src = hist(j, tp, k);
          std::copy(src, src + blk, Gb.begin());
        } else {
          const C* src = hist(tp, j, k);
          for (int c = 0; c < 2; ++c) {
            adjoint(nb, src + c * nbb, &Gb[c * nbb]);
            for (int i = 0; i < nbb; ++i) Gb[c * nbb + i] = -Gb[c * nbb + i];
          }
        }
        const C* S = sig + ((size_t)j * nk + k) * blk;  // Sigma(t_m, t_j)
        for (int i = 0; i < nbb; ++i) {
          SR[i] = S[nbb + i] - S[i];
          GR[i] = Gb[nbb + i] - Gb[i];
        }
        double w1 = quad_weight(p, j, m) * dt;
        double w2 = (j <= tp) ? quad_weight(p, j, tp) * dt : 0.0;
        for (int c = 0; c < 2; ++c) {
          if (w1 != 0.0) {
            mm(nb, SR.data(), &Gb[c * nbb], tmp.data());
            for (int i = 0; i < nbb; ++i) acc[c * nbb + i] += tmp[i] * w1;
          }
          if (w2 != 0.0) {
            mm(nb, S + c * nbb, GR.data(), tmp.data());
            for (int i = 0; i < nbb; ++i) acc[c * nbb + i] -= tmp[i] * w2;
          }
        }
      }
      std::copy(acc.begin(), acc.end(), Iout + ((size_t)tp * nk + k) * blk);
    }
  }
}

// ---------------------------------------------------------------- propagators
// For the midpoint Hamiltonian hbar of one step:
//   V = e^{-i hbar dt},  Vh = e^{-i hbar dt/2},  Phi = (V - 1) hbar^{-1} = -i dt phi1(-i hbar dt),
// so that y(dt) = V y(0) + Phi f solves i dy/dt = hbar y + f exactly for constant f.
// Computed from the spectral decomposition of hbar.
template <class R>
void propagators(int nb, double dt, const Cx<R>* hbar, Cx<R>* V, Cx<R>* Vh, Cx<R>* Phi) {
  typedef Cx<R> C;
  matfun(nb, hbar, [&](R e) { return cexpi(-e * dt); }, V);
  matfun(nb, hbar, [&](R e) { return cexpi(-e * (dt * 0.5)); }, Vh);
  matfun(nb, hbar, [&](R e) {
    // -i dt sum_n z^n/(n+1)!,  z = -i e dt
    C z(R(0.0), -e * dt);
    if (std::fabs(val(e) * dt) < 1.0) {
      C term(1.0), s(1.0);
      for (int n = 1; n < 30; ++n) {
        term = term * z * (1.0 / (n + 1));
        s += term;
      }
      return C(R(0.0), R(-dt)) * s;
    }
    return scale(cexpi(-e * dt) - C(1.0), R(1.0) / e);
  }, Phi);
}

// ---------------------------------------------------------------- observables
template <class R>
void observables(State<R>& st, int m, R* o) {
  typedef Cx<R> C;
  const Params& p = st.p;
  const Grid& g = st.g;
  int nb = g.nb, nbb = st.nbb, nk = g.nk;
  double t = m * p.dt, s = p.spin_deg;
  R A = pulse_A(p, st.th, t);
  std::vector<C> h(nbb), v(nbb), hf(nbb), U(nbb);
  std::vector<R> w(nb);
  hf_field(p, st.th, g, st.rho_cur, hf.data());
  R N = 0.0, Ekin = 0.0, Ehf = 0.0, Ecorr = 0.0, J[2] = {0.0, 0.0};
  std::vector<R> norb(nb, R(0.0)), nband(nb, R(0.0));
  for (int k = 0; k < nk; ++k) {
    const C* r = &st.rho_cur[k * nbb];
    h0(p, g, st.hop.data(), k, A, h.data());
    for (int a = 0; a < nb; ++a) {
      N += r[a * nb + a].re;
      norb[a] += r[a * nb + a].re;
      for (int b = 0; b < nb; ++b) {
        Ekin += (h[a * nb + b] * r[b * nb + a]).re;
        Ehf += (hf[a * nb + b] * r[b * nb + a]).re;
      }
    }
    // E_corr from the equal-time collision integral I^<(t,t) (Galitskii-Migdal form)
    const C* Ik = &st.I_cur[((size_t)m * nk + k) * st.blk];
    for (int a = 0; a < nb; ++a) Ecorr += (C(R(0.0), R(-0.5)) * Ik[a * nb + a]).re;
    for (int d = 0; d < 2; ++d) {
      vel(p, g, st.hop.data(), k, A, d, v.data());
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) J[d] += (v[a * nb + b] * r[b * nb + a]).re;
    }
    eigh(nb, h.data(), w.data(), U.data());
    for (int bnd = 0; bnd < nb; ++bnd) {
      C sacc;
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) sacc += conj(U[a * nb + bnd]) * r[a * nb + b] * U[b * nb + bnd];
      nband[bnd] += sacc.re;
    }
  }
  // the interband preset's one-body -U n_c term is part of the single-particle energy
  std::vector<C> ob(nbb);
  onebody_extra(p, st.th, nb, ob.data());
  for (int k = 0; k < nk; ++k)
    for (int a = 0; a < nb; ++a)
      for (int b = 0; b < nb; ++b) Ekin += (ob[a * nb + b] * st.rho_cur[k * nbb + b * nb + a]).re;
  double inv = 1.0 / nk;
  for (int i = 0; i < NOBS; ++i) o[i] = R(0.0);
  o[OBS_T] = t;
  o[OBS_N] = N * (s * inv);
  o[OBS_EKIN] = Ekin * (s * inv);
  o[OBS_EHF] = Ehf * (0.5 * s * inv);
  o[OBS_ECORR] = Ecorr * (s * inv);
  o[OBS_ETOT] = o[OBS_EKIN] + o[OBS_EHF] + o[OBS_ECORR];
  o[OBS_JX] = J[0] * (s * inv);
  o[OBS_JY] = J[1] * (s * inv);
  o[OBS_A] = A;
  for (int a = 0; a < nb && a < 4; ++a) o[OBS_NORB + a] = norb[a] * inv;
  for (int b = 0; b < nb && b < 4; ++b) o[OBS_NBAND + b] = nband[b] * inv;
}

// ---------------------------------------------------------------- time step
// One step m-1 -> m of Algorithm "prop" (fixed number K of corrector passes), with
// eq. (Green) solved by the exponential midpoint rule:
//   G(t_m, t') = V G(t_{m-1}, t') + Phi Ibar(t'),   t' < t_m,
//   rho_m      = V rho_{m-1} V^dag - dt Vh Dbar Vh^dag,
// where Ibar = I(t_{m-1},.) (predictor) or (I(t_{m-1},.) + I(t_m,.))/2 (corrector),
// Dbar the same average of D = I^<(t,t) + I^<(t,t)^dag (the equal-time form of
// eq. (Green)), and hbar = h0(k - A(t_{m-1/2})) + Sigma^HF[rho] with rho = rho_{m-1}
// (predictor) or (rho_{m-1} + rho_m)/2 (corrector). After the last corrector pass
// Sigma and I are evaluated once more on the accepted row; they feed the next
// step's predictor (the algorithm's "Evaluate ... I(t_{n_t-1}, .)").
template <class R>
void sigma_and_collision(State<R>& st, int m) {
  typedef Cx<R> C;
  int nk = st.g.nk, blk = st.blk;
  std::vector<C> row((size_t)(m + 1) * nk * blk);
  std::copy(st.rows[m].begin(), st.rows[m].end(), row.begin());
  st.sig.assign((size_t)(m + 1) * nk * blk, C());
  sigma_row(st.p, st.th, st.g, m, row.data(), st.sig.data());
  st.I_cur.assign((size_t)(m + 1) * nk * blk, C());
  collision_row<R>(st.p, st.g, m, [&](int j, int tp, int k) { return (const C*)st.at(j, tp, k); },
                   st.sig.data(), st.I_cur.data());
  int nb = st.g.nb, nbb = st.nbb;
  st.D_cur.assign(nk * nbb, C());
  for (int k = 0; k < nk; ++k) {
    const C* Ik = &st.I_cur[((size_t)m * nk + k) * blk];
    for (int a = 0; a < nb; ++a)
      for (int b = 0; b < nb; ++b) st.D_cur[k * nbb + a * nb + b] = Ik[a * nb + b] + conj(Ik[b * nb + a]);
  }
}

template <class R>
void update_row(State<R>& st, int m, bool corrector) {
  typedef Cx<R> C;
  const Params& p = st.p;
  const Grid& g = st.g;
  int nb = g.nb, nbb = st.nbb, blk = st.blk, nk = g.nk;
  std::vector<C> rho_h(nk * nbb);
  for (int i = 0; i < nk * nbb; ++i)
    rho_h[i] = corrector ? (st.rho_prev[i] + st.rho_cur[i]) * 0.5 : st.rho_prev[i];
  std::vector<C> hf(nbb), ob(nbb);
  hf_field(p, st.th, g, rho_h, hf.data());
  onebody_extra(p, st.th, nb, ob.data());
  for (int i = 0; i < nbb; ++i) hf[i] += ob[i];
  R Amid = pulse_A(p, st.th, (m - 0.5) * p.dt);
  std::vector<C> new_rho(nk * nbb);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nk; ++k) {
    std::vector<C> h(nbb), V(nbb), Vh(nbb), Phi(nbb), Ib(blk), t1(nbb), t2(nbb), t3(nbb), adj(nbb);
    h0(p, g, st.hop.data(), k, Amid, h.data());
    for (int i = 0; i < nbb; ++i) h[i] += hf[i];
    propagators(nb, p.dt, h.data(), V.data(), Vh.data(), Phi.data());
    for (int tp = 0; tp < m; ++tp) {
      const C* Ip = &st.I_prev[((size_t)tp * nk + k) * blk];
      for (int i = 0; i < blk; ++i)
        Ib[i] = corrector ? (Ip[i] + st.I_cur[((size_t)tp * nk + k) * blk + i]) * 0.5 : Ip[i];
      const C* Gold = st.at(m - 1, tp, k);
      C* Gnew = st.at(m, tp, k);
      for (int c = 0; c < 2; ++c) {
        mm(nb, V.data(), Gold + c * nbb, t1.data());
        mm(nb, Phi.data(), &Ib[c * nbb], t2.data());
        for (int i = 0; i < nbb; ++i) Gnew[c * nbb + i] = t1[i] + t2[i];
      }
    }
    // density matrix
    std::vector<C> Db(nbb);
    for (int i = 0; i < nbb; ++i)
      Db[i] = corrector ? (st.D_prev[k * nbb + i] + st.D_cur[k * nbb + i]) * 0.5 : st.D_prev[k * nbb + i];
    mm(nb, V.data(), &st.rho_prev[k * nbb], t1.data());
    adjoint(nb, V.data(), adj.data());
    mm(nb, t1.data(), adj.data(), t2.data());
    mm(nb, Vh.data(), Db.data(), t1.data());
    adjoint(nb, Vh.data(), adj.data());
    mm(nb, t1.data(), adj.data(), t3.data());
    for (int i = 0; i < nbb; ++i) new_rho[k * nbb + i] = t2[i] - t3[i] * p.dt;
  }
  st.rho_cur = new_rho;
  for (int k = 0; k < nk; ++k) set_diag_block(nb, &st.rho_cur[k * nbb], st.at(m, m, k));
}

// Largest modulus of the change of row m between two iterates (every t', k, component and
// orbital pair, the equal-time block included): the norm of the stopping test of
// Algorithm "prop", which the paper leaves unspecified.
template <class R>
double row_change(const std::vector<Cx<R>>& a, const std::vector<Cx<R>>& b) {
  double mx = 0.0;
  for (size_t i = 0; i < a.size(); ++i) {
    double dr = val(a[i].re) - val(b[i].re), di = val(a[i].im) - val(b[i].im);
    mx = std::max(mx, std::sqrt(dr * dr + di * di));
  }
  return mx;
}

// One step of Algorithm "prop": predictor, then at most n_corr corrector passes; with
// corr_tol > 0 the passes stop at the first whose change of the row is <= corr_tol (the
// algorithm's max and epsilon), otherwise all n_corr passes run. When the loop ends on its
// pass limit with the last change still above corr_tol (the algorithm leaves its loop without
// reaching epsilon), the step is kept and marked as not converged.
template <class R>
void step(State<R>& st, int m) {
  int nk = st.g.nk, blk = st.blk;
  st.rows.emplace_back((size_t)(m + 1) * nk * blk);
  update_row(st, m, false);
  int passes = 0;
  bool reached = st.p.corr_tol <= 0.0;
  for (int it = 0; it < st.p.n_corr; ++it) {
    std::vector<Cx<R>> before;
    if (st.p.corr_tol > 0.0) before = st.rows[m];
    sigma_and_collision(st, m);
    update_row(st, m, true);
    ++passes;
    if (st.p.corr_tol > 0.0) {
      double ch = row_change(st.rows[m], before);
      st.changes.push_back(ch);
      if (ch <= st.p.corr_tol) {
        reached = true;
        break;
      }
    }
  }
  if ((int)st.passes.size() <= m) st.passes.resize(m + 1, 0);
  st.passes[m] = passes;
  if ((int)st.unconverged.size() <= m) st.unconverged.resize(m + 1, 0);
  st.unconverged[m] = (st.p.corr_tol > 0.0 && st.p.n_corr > 0 && !reached) ? 1 : 0;
  sigma_and_collision(st, m);
  st.I_prev = st.I_cur;
  st.D_prev = st.D_cur;
  st.rho_prev = st.rho_cur;
}

// The kick of the dipole pulse on the completed slice m = m0: G(t_m, t') <- K G(t_m, t') for
// t' < m and K G K^dag on the equal-time block (both components), rho_m <- K rho_m K^dag, then
// the self-energy and the collision integrals of the kicked slice (they feed the next step's
// predictor; at m = 0 the integrals are empty).
template <class R>
void dipole_kick(State<R>& st, int m) {
  typedef Cx<R> C;
  if (st.p.pulse_kind != PULSE_DIPOLE_KICK || m != kick_slice(st.p)) return;
  int nb = st.g.nb, nbb = st.nbb, nk = st.g.nk;
  std::vector<C> K(nbb), Kd(nbb), t1(nbb), t2(nbb);
  kick_matrix(st.th, K.data());
  adjoint(nb, K.data(), Kd.data());
  for (int tp = 0; tp <= m; ++tp)
    for (int k = 0; k < nk; ++k)
      for (int c = 0; c < 2; ++c) {
        C* G = st.at(m, tp, k) + c * nbb;
        mm(nb, K.data(), G, t1.data());
        if (tp == m) {
          mm(nb, t1.data(), Kd.data(), t2.data());
          std::copy(t2.begin(), t2.end(), G);
        } else {
          std::copy(t1.begin(), t1.end(), G);
        }
      }
  for (int k = 0; k < nk; ++k) {
    mm(nb, K.data(), &st.rho_cur[k * nbb], t1.data());
    mm(nb, t1.data(), Kd.data(), &st.rho_cur[k * nbb]);
  }
  if (m > 0) sigma_and_collision(st, m);
  st.I_prev = st.I_cur;
  st.D_prev = st.D_cur;
  st.rho_prev = st.rho_cur;
}

template <class R>
void init(State<R>& st) {
  typedef Cx<R> C;
  int nk = st.g.nk, nbb = st.nbb, blk = st.blk;
  std::vector<Cx<double>> hopd(st.hop.size()), rho0;
  for (size_t i = 0; i < hopd.size(); ++i) hopd[i] = Cx<double>(val(st.hop[i].re), val(st.hop[i].im));
  initial_state(st.p, st.g, hopd.data(), rho0);
  st.rho_cur.assign(rho0.size(), C());
  for (size_t i = 0; i < rho0.size(); ++i) st.rho_cur[i] = C(R(rho0[i].re), R(rho0[i].im));
  st.rows.clear();
  st.rows.emplace_back((size_t)nk * blk);
  for (int k = 0; k < nk; ++k) set_diag_block(st.g.nb, &st.rho_cur[k * nbb], st.at(0, 0, k));
  st.rho_prev = st.rho_cur;
  sigma_and_collision(st, 0);  // I(t_0, t_0) = 0: both integrals are empty
  st.I_prev = st.I_cur;
  st.D_prev = st.D_cur;
}

typedef Cx<double> C;

// ---------------------------------------------------------------- full-square propagation
// Test-only mode that pins the symmetry G^{<,>}(t,t')^dag = -G^{<,>}(t',t): the upper triangle
// G(t_j, t_m), j < m, is NOT taken from the lower one but propagated on its own with the
// adjoint (t'-derivative) equation of motion,
//   -i d/dt' G(t,t') = G(t,t') h(t') + I_R(t,t'),
//   I_R^{<,>}(t,t') = int_0^t dtb G^R(t,tb) Sigma^{<,>}(tb,t') + int_0^t' dtb G^{<,>}(t,tb) Sigma^A(tb,t'),
// in the same exponential midpoint form, G(t_j, t_m) = G(t_j, t_{m-1}) V^dag + Ibar_R Phi^dag, with
// its own self-energy column Sigma(t_j, t_m) (forward line from the upper triangle, backward
// line from the lower). Both triangles feed each other's collision integrals and self-energies;
// the diagonal follows the density matrix as in the plain scheme.

// Right-form collision integrals of column m: IR[j] = I_R(t_j, t_m), j = 0..m, with the
// weights of quad_weight; Gat(i, j, k) gives G(t_i, t_j) for any pair; sigcol[l] = Sigma(t_l, t_m).
template <class GA>
void collision_col(const Params& p, const Grid& g, int m, GA Gat, const C* sigcol, C* IR) {
  int nb = g.nb, nbb = nb * nb, blk = 2 * nbb, nk = g.nk;
  double dt = p.dt;
#pragma omp parallel for schedule(dynamic)
  for (int k = 0; k < nk; ++k) {
    std::vector<C> GR(nbb), SR(nbb), tmp(nbb), acc(blk);
    for (int j = 0; j <= m; ++j) {
      std::fill(acc.begin(), acc.end(), C());
      // int_0^{t_j} G^R(t_j, t_l) Sigma^{<,>}(t_l, t_m),  G^R = G^> - G^< (t_l < t_j)
      for (int l = 0; l <= j; ++l) {
        double w = quad_weight(p, l, j) * dt;
        if (w == 0.0) continue;
        const C* G = Gat(j, l, k);
        for (int i = 0; i < nbb; ++i) GR[i] = G[nbb + i] - G[i];
        const C* S = sigcol + ((size_t)l * nk + k) * blk;
        for (int c = 0; c < 2; ++c) {
          mm(nb, GR.data(), S + c * nbb, tmp.data());
          for (int i = 0; i < nbb; ++i) acc[c * nbb + i] += tmp[i] * w;
        }
      }
      // int_0^{t_m} G^{<,>}(t_j, t_l) Sigma^A(t_l, t_m),  Sigma^A = -(Sigma^> - Sigma^<) (t_l < t_m)
      for (int l = 0; l <= m; ++l) {
        double w = quad_weight(p, l, m) * dt;
        if (w == 0.0) continue;
        const C* G = Gat(j, l, k);
        const C* S = sigcol + ((size_t)l * nk + k) * blk;
        for (int i = 0; i < nbb; ++i) SR[i] = S[nbb + i] - S[i];
        for (int c = 0; c < 2; ++c) {
          mm(nb, G + c * nbb, SR.data(), tmp.data());
          for (int i = 0; i < nbb; ++i) acc[c * nbb + i] -= tmp[i] * w;
        }
      }
      std::copy(acc.begin(), acc.end(), IR + ((size_t)j * nk + k) * blk);
    }
  }
}

struct FullSquare {
  Params p;
  Grid g;
  Theta<double> th;
  std::vector<C> hop;
  int n, nk, nb, nbb, blk;
  std::vector<C> G;  // [(i * (n + 1) + j) * nk + k][blk] = G(k; t_i, t_j)
  std::vector<C> rho_prev, rho_cur, D_prev, D_cur;
  std::vector<C> I_prev, I_cur;    // rows:    [t'][k][blk] = I(t_m, t')
  std::vector<C> IR_prev, IR_cur;  // columns: [j][k][blk]  = I_R(t_j, t_m)
  FullSquare(const Params& p_, const double* hopd, int nsteps)
      : p(p_), g(p_), th{p_.amp, p_.omega, p_.U}, n(nsteps) {
    nk = g.nk;
    nb = g.nb;
    nbb = nb * nb;
    blk = 2 * nbb;
    hop.resize(3 * nbb);
    for (int i = 0; i < 3 * nbb; ++i) hop[i] = C(hopd[2 * i], hopd[2 * i + 1]);
    G.assign((size_t)(n + 1) * (n + 1) * nk * blk, C());
  }
  C* at(int i, int j, int k) { return &G[(((size_t)i * (n + 1) + j) * nk + k) * blk]; }
  void eval(int m) {
    size_t sz = (size_t)(m + 1) * nk * blk;
    std::vector<C> fwd(sz), bwd(sz), sr(sz), sc(sz);
    for (int j = 0; j <= m; ++j)
      for (int k = 0; k < nk; ++k) {
        std::copy(at(m, j, k), at(m, j, k) + blk, &fwd[((size_t)j * nk + k) * blk]);
        std::copy(at(j, m, k), at(j, m, k) + blk, &bwd[((size_t)j * nk + k) * blk]);
      }
    sigma_pairs(p, th, g, m, fwd.data(), bwd.data(), sr.data());  // Sigma(t_m, t_j)
    sigma_pairs(p, th, g, m, bwd.data(), fwd.data(), sc.data());  // Sigma(t_j, t_m)
    I_cur.assign(sz, C());
    collision_row<double>(p, g, m, [&](int j, int tp, int k) { return (const C*)at(j, tp, k); }, sr.data(),
                          I_cur.data(), true);
    IR_cur.assign(sz, C());
    collision_col(p, g, m, [&](int i, int j, int k) { return (const C*)at(i, j, k); }, sc.data(), IR_cur.data());
    D_cur.assign(nk * nbb, C());
    for (int k = 0; k < nk; ++k) {
      const C* Ik = &I_cur[((size_t)m * nk + k) * blk];
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) D_cur[k * nbb + a * nb + b] = Ik[a * nb + b] + conj(Ik[b * nb + a]);
    }
  }
  void update(int m, bool corrector) {
    std::vector<C> rho_h(nk * nbb);
    for (int i = 0; i < nk * nbb; ++i) rho_h[i] = corrector ? (rho_prev[i] + rho_cur[i]) * 0.5 : rho_prev[i];
    std::vector<C> hf(nbb), ob(nbb);
    hf_field(p, th, g, rho_h, hf.data());
    onebody_extra(p, th, nb, ob.data());
    for (int i = 0; i < nbb; ++i) hf[i] += ob[i];
    double Amid = pulse_A(p, th, (m - 0.5) * p.dt);
    std::vector<C> new_rho(nk * nbb);
    for (int k = 0; k < nk; ++k) {
      std::vector<C> h(nbb), V(nbb), Vh(nbb), Phi(nbb), Vd(nbb), Phid(nbb), Ib(blk), t1(nbb), t2(nbb), t3(nbb),
          adj(nbb);
      h0(p, g, hop.data(), k, Amid, h.data());
      for (int i = 0; i < nbb; ++i) h[i] += hf[i];
      propagators(nb, p.dt, h.data(), V.data(), Vh.data(), Phi.data());
      adjoint(nb, V.data(), Vd.data());
      adjoint(nb, Phi.data(), Phid.data());
      for (int t = 0; t < m; ++t) {
        // row: G(t_m, t) = V G(t_{m-1}, t) + Phi Ibar(t)
        for (int i = 0; i < blk; ++i) {
          C a = I_prev[((size_t)t * nk + k) * blk + i];
          Ib[i] = corrector ? (a + I_cur[((size_t)t * nk + k) * blk + i]) * 0.5 : a;
        }
        for (int c = 0; c < 2; ++c) {
          mm(nb, V.data(), at(m - 1, t, k) + c * nbb, t1.data());
          mm(nb, Phi.data(), &Ib[c * nbb], t2.data());
          for (int i = 0; i < nbb; ++i) at(m, t, k)[c * nbb + i] = t1[i] + t2[i];
        }
        // column: G(t, t_m) = G(t, t_{m-1}) V^dag + IbarR(t) Phi^dag
        for (int i = 0; i < blk; ++i) {
          C a = IR_prev[((size_t)t * nk + k) * blk + i];
          Ib[i] = corrector ? (a + IR_cur[((size_t)t * nk + k) * blk + i]) * 0.5 : a;
        }
        for (int c = 0; c < 2; ++c) {
          mm(nb, at(t, m - 1, k) + c * nbb, Vd.data(), t1.data());
          mm(nb, &Ib[c * nbb], Phid.data(), t2.data());
          for (int i = 0; i < nbb; ++i) at(t, m, k)[c * nbb + i] = t1[i] + t2[i];
        }
      }
      std::vector<C> Db(nbb);
      for (int i = 0; i < nbb; ++i) Db[i] = corrector ? (D_prev[k * nbb + i] + D_cur[k * nbb + i]) * 0.5 : D_prev[k * nbb + i];
      mm(nb, V.data(), &rho_prev[k * nbb], t1.data());
      mm(nb, t1.data(), Vd.data(), t2.data());
      mm(nb, Vh.data(), Db.data(), t1.data());
      adjoint(nb, Vh.data(), adj.data());
      mm(nb, t1.data(), adj.data(), t3.data());
      for (int i = 0; i < nbb; ++i) new_rho[k * nbb + i] = t2[i] - t3[i] * p.dt;
    }
    rho_cur = new_rho;
    for (int k = 0; k < nk; ++k) set_diag_block(nb, &rho_cur[k * nbb], at(m, m, k));
  }
  void run() {
    std::vector<C> rho0;
    initial_state(p, g, hop.data(), rho0);
    rho_cur = rho0;
    for (int k = 0; k < nk; ++k) set_diag_block(nb, &rho_cur[k * nbb], at(0, 0, k));
    rho_prev = rho_cur;
    eval(0);
    I_prev = I_cur;
    IR_prev = IR_cur;
    D_prev = D_cur;
    for (int m = 1; m <= n; ++m) {
      update(m, false);
      for (int it = 0; it < p.n_corr; ++it) {
        eval(m);
        update(m, true);
      }
      eval(m);
      I_prev = I_cur;
      IR_prev = IR_cur;
      D_prev = D_cur;
      rho_prev = rho_cur;
    }
  }
};

typedef Cx<double> C;

void to_doubles(const C* src, size_t n, double* dst) {
  for (size_t i = 0; i < n; ++i) { dst[2 * i] = src[i].re; dst[2 * i + 1] = src[i].im; }
}
void from_doubles(const double* src, size_t n, C* dst) {
  for (size_t i = 0; i < n; ++i) dst[i] = C(src[2 * i], src[2 * i + 1]);
}

}  // namespace

static int g_progress = 0;

static void report_step(int m, int nsteps) {
  if (g_progress > 0 && (m % g_progress == 0 || m == nsteps)) {
    std::fprintf(stderr, "[oracle] step %d of %d\n", m, nsteps);
    std::fflush(stderr);
  }
}

extern "C" {

int oracle_nobs() { return NOBS; }

// Quadrature weights of eq. (CI) on [0, N]: out[j] = weight of node j, j = 0..N.
// Threads of the OpenMP loops over k: the count the next run uses, and a way to change it (for
// a one-core timing).
int oracle_max_threads() { return omp_get_max_threads(); }
void oracle_set_threads(int32_t n) {
  if (n > 0) omp_set_num_threads(n);
}
// every > 0: the run entry points print "[oracle] step m of n" to stderr after every `every`
// steps (long timing runs); 0 (the default) prints nothing
void oracle_set_progress(int32_t every) { g_progress = every > 0 ? every : 0; }

int oracle_quad_weights(int32_t quad_points, int32_t N, double* out) {
  if (quad_points < 1 || quad_points > QUAD_MAX || N < 0 || !out) return -1;
  Params p{};
  p.quad_points = quad_points;
  for (int j = 0; j <= N; ++j) out[j] = quad_weight(p, j, N);
  return 0;
}

// Full propagation: nsteps steps from the initial state. obs: (nsteps+1) x NOBS.
// final_row (optional): row nsteps, [t'][k][comp][a][b] complex (interleaved re/im).
// hist (optional): rows 0..nsteps concatenated in the same per-row layout.
// rho_out (optional): final rho [k][a][b].
int oracle_run(const Params* p, const double* hop, int32_t nsteps, double* obs, double* final_row,
               double* hist, double* rho_out) {
  if (!p || !hop || nsteps < 0 || p->nb < 1 || p->nb > 4) return -1;
  if (p->interaction == INT_INTERBAND && p->nb != 2) return -1;
  if (p->pulse_kind != PULSE_PEIERLS && (p->pulse_kind != PULSE_DIPOLE_KICK || p->nb != 2 || !(p->t0 >= 0.0)))
    return -1;
  Theta<double> th{p->amp, p->omega, p->U};
  State<double> st(*p, th, hop);
  init(st);
  if (obs) observables(st, 0, obs);
  dipole_kick(st, 0);
  for (int m = 1; m <= nsteps; ++m) {
    step(st, m);
    if (obs) observables(st, m, obs + (size_t)m * NOBS);
    dipole_kick(st, m);
    report_step(m, nsteps);
  }
  if (final_row) to_doubles(st.rows[nsteps].data(), st.rows[nsteps].size(), final_row);
  if (hist) {
    size_t off = 0;
    for (int j = 0; j <= nsteps; ++j) {
      to_doubles(st.rows[j].data(), st.rows[j].size(), hist + 2 * off);
      off += st.rows[j].size();
    }
  }
  if (rho_out) to_doubles(st.rho_cur.data(), st.rho_cur.size(), rho_out);
  return 0;
}

// oracle_run with the corrector log: passes[m] = corrector passes of step m (passes[0] = 0);
// changes[(m - 1) * n_corr + i] = row change after pass i of step m (-1 where no pass ran;
// only filled when corr_tol > 0); unconverged[m] = 1 where step m ran all n_corr passes and
// its last change was still above corr_tol.
int oracle_run_log(const Params* p, const double* hop, int32_t nsteps, double* obs, int32_t* passes,
                   double* changes, int32_t* unconverged) {
  if (!p || !hop || nsteps < 0 || p->nb < 1 || p->nb > 4) return -1;
  if (p->interaction == INT_INTERBAND && p->nb != 2) return -1;
  if (p->pulse_kind != PULSE_PEIERLS && (p->pulse_kind != PULSE_DIPOLE_KICK || p->nb != 2 || !(p->t0 >= 0.0)))
    return -1;
  Theta<double> th{p->amp, p->omega, p->U};
  State<double> st(*p, th, hop);
  init(st);
  if (obs) observables(st, 0, obs);
  dipole_kick(st, 0);
  if (changes)
    for (int64_t i = 0; i < (int64_t)nsteps * p->n_corr; ++i) changes[i] = -1.0;
  for (int m = 1; m <= nsteps; ++m) {
    size_t c0 = st.changes.size();
    step(st, m);
    if (obs) observables(st, m, obs + (size_t)m * NOBS);
    dipole_kick(st, m);
    if (changes)
      for (size_t i = c0; i < st.changes.size(); ++i) changes[(size_t)(m - 1) * p->n_corr + (i - c0)] = st.changes[i];
  }
  if (passes)
    for (int m = 0; m <= nsteps; ++m) passes[m] = m < (int)st.passes.size() ? st.passes[m] : 0;
  if (unconverged)
    for (int m = 0; m <= nsteps; ++m) unconverged[m] = m < (int)st.unconverged.size() ? st.unconverged[m] : 0;
  return 0;
}

// Tangent-linear run: the same propagation in Dual<3> arithmetic, seeded with the unit
// directions of (pulse amplitude, pulse frequency, U). obs: (nsteps+1) x NOBS values,
// dobs: (nsteps+1) x NOBS x 3 derivatives d obs / d(amp, omega, U).
int oracle_tlm_run(const Params* p, const double* hop, int32_t nsteps, double* obs, double* dobs) {
  if (!p || !hop || nsteps < 0 || p->nb < 1 || p->nb > 4) return -1;
  if (p->interaction == INT_INTERBAND && p->nb != 2) return -1;
  if (p->pulse_kind != PULSE_PEIERLS && (p->pulse_kind != PULSE_DIPOLE_KICK || p->nb != 2 || !(p->t0 >= 0.0)))
    return -1;
  Theta<D3> th;
  th.amp = D3(p->amp);
  th.amp.d[0] = 1.0;
  th.omega = D3(p->omega);
  th.omega.d[1] = 1.0;
  th.U = D3(p->U);
  th.U.d[2] = 1.0;
  State<D3> st(*p, th, hop);
  init(st);
  std::vector<D3> o(NOBS);
  auto emit = [&](int m) {
    observables(st, m, o.data());
    for (int i = 0; i < NOBS; ++i) {
      if (obs) obs[(size_t)m * NOBS + i] = o[i].v;
      if (dobs)
        for (int q = 0; q < 3; ++q) dobs[((size_t)m * NOBS + i) * 3 + q] = o[i].d[q];
    }
  };
  emit(0);
  dipole_kick(st, 0);
  for (int m = 1; m <= nsteps; ++m) {
    step(st, m);
    emit(m);
    dipole_kick(st, m);
    report_step(m, nsteps);
  }
  return 0;
}

// Sigma on row m: row and out are [j=0..m][k][comp][a][b] complex.
int oracle_sigma_row(const Params* p, int32_t m, const double* row, double* out) {
  Grid g(*p);
  Theta<double> th{p->amp, p->omega, p->U};
  size_t n = (size_t)(m + 1) * g.nk * 2 * g.nb * g.nb;
  std::vector<C> r(n), o(n);
  from_doubles(row, n, r.data());
  sigma_row(*p, th, g, m, r.data(), o.data());
  to_doubles(o.data(), n, out);
  return 0;
}

// Collision integrals I(t_m, t'), t' = 0..m. hist: rows 0..m concatenated
// (row j = [t'=0..j][k][comp][a][b]); sig: [j][k][comp][a][b]; out: [t'][k][comp][a][b].
int oracle_collision_row(const Params* p, int32_t m, const double* hist, const double* sig, double* out) {
  Grid g(*p);
  int blk = 2 * g.nb * g.nb, nk = g.nk;
  std::vector<size_t> rowoff(m + 2, 0);
  for (int j = 0; j <= m; ++j) rowoff[j + 1] = rowoff[j] + (size_t)(j + 1) * nk * blk;
  std::vector<C> H(rowoff[m + 1]), S((size_t)(m + 1) * nk * blk), O((size_t)(m + 1) * nk * blk);
  from_doubles(hist, H.size(), H.data());
  from_doubles(sig, S.size(), S.data());
  collision_row<double>(*p, g, m,
                        [&](int j, int tp, int k) { return (const C*)&H[rowoff[j] + ((size_t)tp * nk + k) * blk]; },
                        S.data(), O.data());
  to_doubles(O.data(), O.size(), out);
  return 0;
}

// V, Vh, Phi for a batch of Hermitian matrices hbar: [count][a][b] -> out [count][3][a][b].
int oracle_propagators(int32_t nb, int32_t count, double dt, const double* hbar, double* out) {
  int nbb = nb * nb;
  std::vector<C> h(nbb), V(nbb), Vh(nbb), Phi(nbb);
  for (int i = 0; i < count; ++i) {
    from_doubles(hbar + 2 * (size_t)i * nbb, nbb, h.data());
    propagators(nb, dt, h.data(), V.data(), Vh.data(), Phi.data());
    to_doubles(V.data(), nbb, out + 2 * ((size_t)i * 3 + 0) * nbb);
    to_doubles(Vh.data(), nbb, out + 2 * ((size_t)i * 3 + 1) * nbb);
    to_doubles(Phi.data(), nbb, out + 2 * ((size_t)i * 3 + 2) * nbb);
  }
  return 0;
}

// Eigen-decomposition (ascending) of a batch of Hermitian matrices.
int oracle_eigh(int32_t nb, int32_t count, const double* A, double* w, double* vec) {
  int nbb = nb * nb;
  std::vector<C> a(nbb), v(nbb);
  for (int i = 0; i < count; ++i) {
    from_doubles(A + 2 * (size_t)i * nbb, nbb, a.data());
    eigh(nb, a.data(), w + (size_t)i * nb, v.data());
    to_doubles(v.data(), nbb, vec + 2 * (size_t)i * nbb);
  }
  return 0;
}

// Initial density matrix rho0 [k][a][b] and chemical potential.
int oracle_initial_state(const Params* p, const double* hop, double* rho0, double* mu) {
  Grid g(*p);
  int nbb = g.nb * g.nb;
  std::vector<C> H(3 * nbb);
  from_doubles(hop, 3 * nbb, H.data());
  std::vector<C> rho;
  double m = initial_state(*p, g, H.data(), rho);
  to_doubles(rho.data(), rho.size(), rho0);
  if (mu) *mu = m;
  return 0;
}

// h0(k - A pol) for every k: out [k][a][b].
int oracle_h0(const Params* p, const double* hop, double A, double* out) {
  Grid g(*p);
  int nbb = g.nb * g.nb;
  std::vector<C> H(3 * nbb), h(nbb);
  from_doubles(hop, 3 * nbb, H.data());
  for (int k = 0; k < g.nk; ++k) {
    h0(*p, g, H.data(), k, A, h.data());
    to_doubles(h.data(), nbb, out + 2 * (size_t)k * nbb);
  }
  return 0;
}

// Full-square propagation (test only): out[0] = max |G(t_i,t_j) + G(t_j,t_i)^dag| / max |G| over
// i < j, out[1] = max |rho - rho^dag| over all steps' final rho, out[2] = max relative difference
// of the lower triangle from the plain run's rows (which take the upper triangle as -G^dag).
int oracle_full_square_check(const Params* p, const double* hop, int32_t nsteps, double* out) {
  if (p->nt < nsteps || p->pulse_kind != PULSE_PEIERLS) return -1;
  FullSquare fsq(*p, hop, nsteps);
  fsq.run();
  int nk = fsq.nk, nb = fsq.nb, nbb = fsq.nbb, blk = fsq.blk, n = nsteps;
  double gmax = 0.0, asym = 0.0;
  for (int i = 0; i <= n; ++i)
    for (int j = 0; j <= n; ++j)
      for (int k = 0; k < nk; ++k) {
        const C* a = fsq.at(i, j, k);
        for (int e = 0; e < blk; ++e) gmax = std::max(gmax, std::sqrt(abs2(a[e])));
        if (i >= j) continue;
        const C* b = fsq.at(j, i, k);
        for (int c = 0; c < 2; ++c)
          for (int x = 0; x < nb; ++x)
            for (int y = 0; y < nb; ++y) {
              C d = a[c * nbb + x * nb + y] + conj(b[c * nbb + y * nb + x]);
              asym = std::max(asym, std::sqrt(abs2(d)));
            }
      }
  double herm = 0.0;
  for (int k = 0; k < nk; ++k)
    for (int x = 0; x < nb; ++x)
      for (int y = 0; y < nb; ++y) {
        C d = fsq.rho_cur[k * nbb + x * nb + y] - conj(fsq.rho_cur[k * nbb + y * nb + x]);
        herm = std::max(herm, std::sqrt(abs2(d)));
      }
  // plain run on the same parameters
  Theta<double> th{p->amp, p->omega, p->U};
  State<double> st(*p, th, hop);
  init(st);
  for (int m = 1; m <= n; ++m) step(st, m);
  double diff = 0.0;
  for (int i = 0; i <= n; ++i)
    for (int j = 0; j <= i; ++j)
      for (int k = 0; k < nk; ++k) {
        const C* a = fsq.at(i, j, k);
        const C* b = st.at(i, j, k);
        for (int e = 0; e < blk; ++e) diff = std::max(diff, std::sqrt(abs2(a[e] - b[e])));
      }
  out[0] = asym / gmax;
  out[1] = herm;
  out[2] = diff / gmax;
  return 0;
}

}  // extern "C"
