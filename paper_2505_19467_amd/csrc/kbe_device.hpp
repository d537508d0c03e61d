// Device-side helpers of the gfx950 Kadanoff-Baym library: complex arithmetic on
// double2, small fixed-size matrix products, the packed two-time layout, and the
// single-particle Hamiltonian of the lattice model.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kbe {

typedef double2 cplx;

// ------------------------------------------------------------------ complex arithmetic
__device__ __forceinline__ cplx cmk(double r, double i) { return make_double2(r, i); }
__device__ __forceinline__ cplx czero() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cplx cneg(cplx a) { return make_double2(-a.x, -a.y); }
__device__ __forceinline__ cplx cconj(cplx a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ cplx cscal(cplx a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ cplx cmuli(cplx a) { return make_double2(-a.y, a.x); }  // i * a
// acc += a * b
__device__ __forceinline__ void cmac(cplx& acc, cplx a, cplx b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc += a * conj(b)
__device__ __forceinline__ void cmacc(cplx& acc, cplx a, cplx b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.y, b.x, acc.y);
  acc.y = fma(-a.x, b.y, acc.y);
}
__device__ __forceinline__ double cabs2(cplx a) { return a.x * a.x + a.y * a.y; }

// ------------------------------------------------------------------ NB x NB matrices (row-major)
template <int NB>
__device__ __forceinline__ void mat_zero(cplx* A) {
#pragma unroll
  for (int i = 0; i < NB * NB; ++i) A[i] = czero();
}
// acc += A B
template <int NB>
__device__ __forceinline__ void mm_acc(cplx* acc, const cplx* A, const cplx* B) {
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int l = 0; l < NB; ++l) cmac(acc[i * NB + j], A[i * NB + l], B[l * NB + j]);
}
// acc += A B^dag   ((A B^dag)_ij = sum_l A_il conj(B_jl))
template <int NB>
__device__ __forceinline__ void mm_acc_bdag(cplx* acc, const cplx* A, const cplx* B) {
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int l = 0; l < NB; ++l) cmacc(acc[i * NB + j], A[i * NB + l], B[j * NB + l]);
}

// ------------------------------------------------------------------ layout
// Packed two-time history, strip-major and component-interleaved. Columns t' are grouped in
// strips of 64; strip s stores the rows j = 64 s .. N-1 (N = nt_max + 1) of its columns, and
// each row segment holds the C = 2 nb^2 components one after the other, 64 elements each:
//   elem(k, c, j, t') = k C P + C (base(s) + 64 (j - 64 s)) + 64 c + (t' - 64 s),  s = t' / 64,
//   base(s) = sum_{s' < s} 64 (N - 64 s') = 64 s N - 2048 s (s - 1),  P = base(ceil(N / 64)).
// A strip of one k is a single contiguous run of rows of C x 64 elements, which the history
// sums stream front to back (the entries above the diagonal in a strip's first 64 rows are
// unused). In the FP32 form (complex64 elements) the components of a row segment are stored
// in pairs, interleaved per column, so that one 16-byte load brings a lane two components:
//   elem = k C P + C (base(s) + 64 (j - 64 s)) + 128 (c / 2) + 2 (t' - 64 s) + (c % 2).
__host__ __device__ __forceinline__ int64_t strip_base(int64_t s, int64_t N) { return 64 * s * N - 2048 * s * (s - 1); }

struct Dims {
  int nkx, nky, nk, nb;
  int nbb, C;      // nb^2, 2 nb^2 complex components per two-time block
  int N;           // rows of the history (nt_max + 1)
  int Tp;          // padded length of per-row buffers (>= nt_max + 1, multiple of 8)
  int Smax;        // number of 64-column strips of the largest history pass
  int fp32;        // 1: the packed history is stored in FP32 (complex64)
  int mfma;        // 1: FP32 storage in the quad layout of the matrix-core history sums
  int spb;         // 64-column strips per row-partial slot group: 2 when one history-sum block
                   // covers a pair of strips (nb <= 2), else 1
  int qp;          // quadrature nodes per end carrying end corrections (1: trapezoid)
  int rring;       // FP64 working rows kept (the last rring rows, max(2, qp))
  int64_t P;       // history elements per (k, component): one k occupies C * P elements
};

// Row segment (j, strip of t') of a k, in units of C-component rows of 64 elements.
__host__ __device__ __forceinline__ int64_t seg_off(const Dims& d, int j, int tp) {
  int s = tp >> 6;
  return strip_base(s, d.N) + 64 * (int64_t)(j - 64 * s);
}
// Quad layout of the FP32-MFMA form. Strip s of a k holds its rows j = 64 s .. in quads of 4
// rows (the last quad padded), Q(s) = ceil((N - 64 s) / 4) quads of 4 x 64 x C complex64
// elements each. Inside a quad the 64 columns form 4 groups g of 16; lane L = 16 (j % 4) +
// (t' % 16) of a wavefront holds the (row, column) pair that feeds the matrix cores as their
// K x N operand tile, and the components come in pairs c = 2 ci, 2 ci + 1 (one 16-byte load):
//   elem(k, c, j, t') = k C P + 256 C (qbase(s) + q) + 2 (64 (g C / 2 + ci) + L) + c % 2,
//   q = (j - 64 s) / 4,  qbase(s) = sum_{s' < s} Q(s') = s Qn - 8 s (s - 1),  Qn = ceil(N / 4),
//   P = 256 qbase(ceil(N / 64)).
__host__ __device__ __forceinline__ int64_t quad_base(int64_t s, int64_t N) {
  return s * ((N + 3) / 4) - 8 * s * (s - 1);
}
// Element index (complex units of the storage type).
__host__ __device__ __forceinline__ int64_t hist_idx(const Dims& d, int k, int c, int j, int tp) {
  if (d.mfma) {
    int s = tp >> 6, rel = j - 64 * s;
    int L = 16 * (rel & 3) + (tp & 15), g = (tp >> 4) & 3;
    int64_t seg = quad_base(s, d.N) + (rel >> 2);
    return (int64_t)k * d.C * d.P + 256 * (int64_t)d.C * seg + 2 * (64 * (int64_t)(g * (d.C >> 1) + (c >> 1)) + L) +
           (c & 1);
  }
  int64_t in_seg = d.fp32 ? 128 * (c >> 1) + 2 * (tp & 63) + (c & 1) : 64 * c + (tp & 63);
  return (int64_t)k * d.C * d.P + (int64_t)d.C * seg_off(d, j, tp) + in_seg;
}
// Strip s of k seen from lane `lane`: element (c, j) of the strip is at this + 64 C j + 64 c
// (FP64), or component pair c2 at this + 64 C j + 128 c2 (FP32 form).
__host__ __device__ __forceinline__ int64_t strip_lane_base(const Dims& d, int k, int s, int lane) {
  return (int64_t)k * d.C * d.P + (int64_t)d.C * (strip_base(s, d.N) - 64 * 64 * (int64_t)s) +
         (d.fp32 ? 2 * lane : lane);
}
// FP64 working copies of the last rring history rows: [slot = row % rring][k][C][Tp].
__host__ __device__ __forceinline__ int64_t row64_idx(const Dims& d, int row, int k, int c, int t) {
  return (((int64_t)(row % d.rring) * d.nk + k) * d.C + c) * d.Tp + t;
}
// FP64 copies of history columns 0..qp-1: element (row, col), col < qp, row >= col.
__host__ __device__ __forceinline__ int64_t colq_idx(const Dims& d, int k, int c, int row, int col) {
  return (((int64_t)k * d.C + c) * d.qp + col) * d.Tp + row;
}
// FP64 copies of the history diagonal band: element (row, row - off), off < qp, off <= row.
__host__ __device__ __forceinline__ int64_t band_idx(const Dims& d, int k, int c, int row, int off) {
  return (((int64_t)k * d.C + c) * d.qp + off) * d.Tp + row;
}
// Row-partial sums of the history sums: [k][slot][nb^2][Tp], slot = strip / spb.
__host__ __device__ __forceinline__ const cplx* rowpart_slot(const Dims& d, const cplx* rowpart, int k, int slot) {
  return rowpart + ((int64_t)k * d.Smax + slot) * d.nbb * d.Tp;
}
__host__ __device__ __forceinline__ int64_t rowbuf_idx(const Dims& d, int k, int c, int t) {
  return ((int64_t)k * d.C + c) * d.Tp + t;
}
// Sigma row: [k][3][nb^2][Tp] with components 0: Sigma^<, 1: Sigma^>, 2: Sigma^> - Sigma^<.
__host__ __device__ __forceinline__ int64_t sig_idx(const Dims& d, int k, int s, int e, int t) {
  return (((int64_t)k * 3 + s) * d.nbb + e) * d.Tp + t;
}

// ------------------------------------------------------------------ quadrature of eq. (CI)
// End corrections of the collision-integral quadrature, filled on the host: with q nodes per
// end, node j of [0, N] weighs 1 + c[q'][j] [j < q'] + c[q'][N - j] [N - j < q'],
// q' = min(q, N + 1); q = 1 is the trapezoid rule (c[1][0] = -1/2), N = 0 the empty integral.
constexpr int KBE_QMAX = 6;
struct QuadW {
  int q;
  double c[KBE_QMAX + 1][KBE_QMAX];
};
__host__ __device__ __forceinline__ double quad_w(const QuadW& Q, int j, int N) {
  if (N <= 0) return 0.0;
  int qq = Q.q < N + 1 ? Q.q : N + 1;
  double w = 1.0;
  if (j < qq) w += Q.c[qq][j];
  if (N - j < qq) w += Q.c[qq][N - j];
  return w;
}

// ------------------------------------------------------------------ model
// Bloch Hamiltonian h0(q) = T0 + sum_d [T_d e^{i q_d} + T_d^dag e^{-i q_d}] at q = k - A,
// k from eq. (kj): k_j = -pi + 2 pi j / n. hop = [T0, Tx, Ty], each NB x NB.
template <int NB>
__device__ __forceinline__ void bloch_h0(const cplx* __restrict__ hop, int nkx, int nky, int k, double Ax,
                                         double Ay, cplx* h) {
  int ix = k / nky, iy = k - (k / nky) * nky;
  double qx = -M_PI + 2.0 * M_PI * (double)ix / (double)nkx - Ax;
  double sx, cx;
  sincos(qx, &sx, &cx);
  cplx ex = cmk(cx, sx), emx = cmk(cx, -sx);
  cplx ey = czero(), emy = czero();
  bool two = nky > 1;
  if (two) {
    double qy = -M_PI + 2.0 * M_PI * (double)iy / (double)nky - Ay;
    double sy, cy;
    sincos(qy, &sy, &cy);
    ey = cmk(cy, sy);
    emy = cmk(cy, -sy);
  }
  const cplx* T0 = hop;
  const cplx* Tx = hop + NB * NB;
  const cplx* Ty = hop + 2 * NB * NB;
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      cplx s = T0[a * NB + b];
      s = cadd(s, cmul(Tx[a * NB + b], ex));
      s = cadd(s, cmul(cconj(Tx[b * NB + a]), emx));
      if (two) {
        s = cadd(s, cmul(Ty[a * NB + b], ey));
        s = cadd(s, cmul(cconj(Ty[b * NB + a]), emy));
      }
      h[a * NB + b] = s;
    }
}

// Velocity d h0 / d q_d = i (T_d e^{i q_d} - T_d^dag e^{-i q_d}) at q = k - A.
template <int NB>
__device__ __forceinline__ void bloch_vel(const cplx* __restrict__ hop, int nkx, int nky, int k, double Ax,
                                          double Ay, int dir, cplx* v) {
  int ix = k / nky, iy = k - (k / nky) * nky;
  double q = dir == 0 ? (-M_PI + 2.0 * M_PI * (double)ix / (double)nkx - Ax)
                      : (-M_PI + 2.0 * M_PI * (double)iy / (double)nky - Ay);
  double sq, cq;
  sincos(q, &sq, &cq);
  cplx e = cmk(cq, sq), em = cmk(cq, -sq);
  const cplx* T = hop + (1 + dir) * NB * NB;
  bool on = (dir == 0) || (nky > 1);
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      cplx s = csub(cmul(T[a * NB + b], e), cmul(cconj(T[b * NB + a]), em));
      v[a * NB + b] = on ? cmuli(s) : czero();
    }
}

// Eigen-decomposition of a Hermitian NB x NB matrix held by one thread: cyclic Jacobi
// sweeps with complex plane rotations. A is overwritten; w ascending, columns of V the
// eigenvectors (A_in = V diag(w) V^dag).
template <int NB>
__device__ void jacobi_eigh(cplx* A, double* w, cplx* V) {
#pragma unroll
  for (int i = 0; i < NB * NB; ++i) V[i] = czero();
#pragma unroll
  for (int i = 0; i < NB; ++i) V[i * NB + i] = cmk(1.0, 0.0);
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dia = 0.0;
#pragma unroll
    for (int p = 0; p < NB; ++p)
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        if (p == q) dia += cabs2(A[p * NB + q]);
        else off += cabs2(A[p * NB + q]);
      }
    if (!(off > 1e-34 * (dia + 1e-300))) break;
#pragma unroll
    for (int p = 0; p < NB - 1; ++p)
#pragma unroll
      for (int q = p + 1; q < NB; ++q) {
        cplx apq = A[p * NB + q];
        double r = sqrt(cabs2(apq));
        if (r < 1e-300) continue;
        cplx e = cscal(apq, 1.0 / r);
        double tau = (A[q * NB + q].x - A[p * NB + p].x) / (2.0 * r);
        double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        // plane unitary: col p = (c, -s conj(e)), col q = (s, c conj(e))
        cplx wqp = cscal(cconj(e), -s), wqq = cscal(cconj(e), c);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          cplx aip = A[i * NB + p], aiq = A[i * NB + q];
          A[i * NB + p] = cadd(cscal(aip, c), cmul(aiq, wqp));
          A[i * NB + q] = cadd(cscal(aip, s), cmul(aiq, wqq));
          cplx vip = V[i * NB + p], viq = V[i * NB + q];
          V[i * NB + p] = cadd(cscal(vip, c), cmul(viq, wqp));
          V[i * NB + q] = cadd(cscal(vip, s), cmul(viq, wqq));
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          cplx apj = A[p * NB + j], aqj = A[q * NB + j];
          A[p * NB + j] = cadd(cscal(apj, c), cmul(cconj(wqp), aqj));
          A[q * NB + j] = cadd(cscal(apj, s), cmul(cconj(wqq), aqj));
        }
        A[p * NB + q] = czero();
        A[q * NB + p] = czero();
        A[p * NB + p].y = 0.0;
        A[q * NB + q].y = 0.0;
      }
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) w[i] = A[i * NB + i].x;
  // insertion sort, ascending, carrying the eigenvector columns
  for (int i = 1; i < NB; ++i)
    for (int j = i; j > 0 && w[j - 1] > w[j]; --j) {
      double tw = w[j];
      w[j] = w[j - 1];
      w[j - 1] = tw;
      for (int r = 0; r < NB; ++r) {
        cplx tv = V[r * NB + j];
        V[r * NB + j] = V[r * NB + j - 1];
        V[r * NB + j - 1] = tv;
      }
    }
}

// ------------------------------------------------------------------ block reductions
template <int N>
__device__ __forceinline__ void block_sum_cplx(cplx* v, cplx* lds /* [N][256] */) {
  int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < N; ++i) lds[i * 256 + t] = v[i];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
#pragma unroll
      for (int i = 0; i < N; ++i) lds[i * 256 + t] = cadd(lds[i * 256 + t], lds[i * 256 + t + s]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = lds[i * 256];
  __syncthreads();
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}


// Cross-lane helpers on doubles (two 32-bit halves). gfx950's permlane swaps exchange
// half-waves / 16-lane rows between two registers on the VALU, DPP moves within rows.
__device__ __forceinline__ void dsplit(double x, unsigned& lo, unsigned& hi) {
  unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  lo = (unsigned)u;
  hi = (unsigned)(u >> 32);
}
__device__ __forceinline__ double djoin(unsigned lo, unsigned hi) {
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// a <- [a_lo + a_hi | b_lo + b_hi] over the two half-waves (lanes l and l+32)
__device__ __forceinline__ double rs_half(double a, double b) {
  unsigned al, ah, bl, bh;
  dsplit(a, al, ah);
  dsplit(b, bl, bh);
  auto l = __builtin_amdgcn_permlane32_swap(al, bl, false, false);
  auto h = __builtin_amdgcn_permlane32_swap(ah, bh, false, false);
  return djoin(l[0], h[0]) + djoin(l[1], h[1]);
}
// rows of 16 lanes: a = [a0 a1 a2 a3], b = [b0 b1 b2 b3] -> [a0+a1, b0+b1, a2+a3, b2+b3]
__device__ __forceinline__ double rs_row(double a, double b) {
  unsigned al, ah, bl, bh;
  dsplit(a, al, ah);
  dsplit(b, bl, bh);
  auto l = __builtin_amdgcn_permlane16_swap(al, bl, false, false);
  auto h = __builtin_amdgcn_permlane16_swap(ah, bh, false, false);
  return djoin(l[0], h[0]) + djoin(l[1], h[1]);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  unsigned lo, hi;
  dsplit(x, lo, hi);
  lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)lo, CTRL, 0xF, 0xF, false);
  hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)hi, CTRL, 0xF, 0xF, false);
  return djoin(lo, hi);
}
// sum over the 16 lanes of each row, result in every lane of the row
__device__ __forceinline__ double row16_sum(double x) {
  x += dpp_d<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_d<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_d<0x141>(x);  // row_half_mirror
  x += dpp_d<0x140>(x);  // row_mirror
  return x;
}


// ------------------------------------------------------------------ history streams and row partials
// Compile-time flag for the masked and unmasked copies of a loop body.
template <bool B>
struct BoolTag {
  static constexpr bool value = B;
};
// Compile-time count (e.g. the strips of a pair that have work in a loop body's rows).
template <int N>
struct IntTag {
  static constexpr int value = N;
};

// Keep the compiler from moving LDS accesses of one wavefront across this point (the lanes of
// a wavefront exchange values through LDS; the hardware executes them in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// History blocks are read once per pass: stream them past the caches.
typedef double kbe_d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cplx load_stream(const cplx* p) {
  kbe_d2v v = __builtin_nontemporal_load(reinterpret_cast<const kbe_d2v*>(p));
  return make_double2(v.x, v.y);
}
// Streaming store of one complex value (row partials are not read again in this pass).
__device__ __forceinline__ void store_stream(cplx* p, cplx v) {
  kbe_d2v w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<kbe_d2v*>(p));
}

// Reduce-scatter of the row terms of R rows (R = 1, 2, 4) over the 64 lanes: half-wave and
// 16-lane-row permlane swaps, then DPP within rows. Afterwards rt[0][q] holds whole-row sums
// in the lanes for which reduced_row<R>(lane) >= 0 names the row:
//   R = 4: lanes 0-15 row 0, 32-47 row 1, 16-31 row 2, 48-63 row 3
//   R = 2: lanes 0-31 row 0, 32-63 row 1;   R = 1: every lane row 0
template <int R, int Q>
__device__ __forceinline__ void reduce_rows(double (&rt)[R][Q]) {
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    double y;
    if constexpr (R == 4) {
      y = rs_row(rs_half(rt[0][q], rt[1][q]), rs_half(rt[2][q], rt[3][q]));
    } else if constexpr (R == 2) {
      double x = rs_half(rt[0][q], rt[1][q]);
      y = rs_row(x, x);
    } else {
      double x = rs_half(rt[0][q], rt[0][q]);
      y = rs_row(x, x);
    }
    rt[0][q] = row16_sum(y);
  }
}
// the one lane per row that stores it (-1: none)
template <int R>
__device__ __forceinline__ int reduced_row(int lane) {
  if constexpr (R == 4) {
    return (lane & 15) == 0 ? (((lane >> 5) & 1) | (((lane >> 4) & 1) << 1)) : -1;
  } else if constexpr (R == 2) {
    return (lane & 31) == 0 ? (lane >> 5) : -1;
  } else {
    return lane == 0 ? 0 : -1;
  }
}


// ------------------------------------------------------------------ factorised line transforms

// Roots of unity tw[u] = e^{+2 pi i u / n}, u < n, into an LDS table (the block's threads in turn).
__device__ __forceinline__ void fill_roots(cplx* tw, int n) {
  for (int u = threadIdx.x; u < n; u += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)u / (double)n, &sn, &cs);
    tw[u] = cmk(cs, sn);
  }
}
__device__ __forceinline__ cplx root(const cplx* tw, int u, int sgn) {
  cplx w = tw[u];
  return sgn > 0 ? w : cconj(w);
}
// largest divisor n1 of n with n1 * n1 <= n (1 when n is prime)
__host__ __device__ __forceinline__ int fft_split(int n) {
  int best = 1;
  for (int f = 2; f * f <= n; ++f)
    if (n % f == 0) best = f;
  return best;
}

// In-place DFT of the lines of two arrays held in LDS:
//   x[line][q] <- scale * sum_p x[line][p] w^{sgn p q},  w = e^{2 pi i / n},
// element p of a line at line * line_mul + p * stride; (t0, t1) are scratch of the same shape.
// For n = n1 n2 (n1 = fft_split(n) > 1) in two Cooley-Tukey stages with p = n2 p1 + p2,
// q = q1 + n1 q2: first the n1-point transforms over p1 with the twiddle w^{p2 q1} into the
// scratch, then the n2-point transforms over p2 back into x; each output costs n1 + n2
// multiply-adds instead of n. Horner chains in registers (8 outputs per item), roots from the
// LDS table tw (n entries, fill_roots).
// Every stage ends with a block barrier; the caller synchronises before the first.
__device__ __forceinline__ void axis_dft(cplx* __restrict__ x0, cplx* __restrict__ x1, cplx* __restrict__ t0,
                                         cplx* __restrict__ t1, int n, int nlines, int line_mul, int stride,
                                         const cplx* __restrict__ tw, int sgn, double scale) {
  const int n1 = fft_split(n);
  if (n1 == 1) {
    int items = 2 * nlines * n;
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
      int arr = it / (nlines * n);
      int rem = it - arr * nlines * n;
      int line = rem / n, q = rem - (rem / n) * n;
      const cplx* x = (arr ? x1 : x0) + line * line_mul;
      cplx z = root(tw, q, sgn), acc = czero();
      for (int p = n - 1; p >= 0; --p) acc = cadd(cmul(acc, z), x[p * stride]);
      (arr ? t1 : t0)[line * line_mul + q * stride] = cscal(acc, scale);
    }
    __syncthreads();
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
      int arr = it / (nlines * n);
      int rem = it - arr * nlines * n;
      int line = rem / n, q = rem - (rem / n) * n;
      int o = line * line_mul + q * stride;
      (arr ? x1 : x0)[o] = (arr ? t1 : t0)[o];
    }
    __syncthreads();
    return;
  }
  const int n2 = n / n1;
  constexpr int Q = 8;
  // stage A: item = (array, line, p2, group of 8 q1): Horner chains over p1 read from LDS
  const int groupsA = (n1 + Q - 1) / Q;
  int itemsA = 2 * nlines * n2 * groupsA;
  for (int it = threadIdx.x; it < itemsA; it += blockDim.x) {
    int arr = it / (nlines * n2 * groupsA);
    int rem = it - arr * nlines * n2 * groupsA;
    int line = rem / (n2 * groupsA);
    rem -= line * n2 * groupsA;
    int p2 = rem / groupsA, g = rem - (rem / groupsA) * groupsA;
    const cplx* x = (arr ? x1 : x0) + line * line_mul;
    cplx* t = (arr ? t1 : t0) + line * line_mul;
    cplx z[Q], acc[Q];
#pragma unroll
    for (int r = 0; r < Q; ++r) {
      int q1 = g * Q + r;
      z[r] = root(tw, ((q1 < n1 ? q1 : 0) * n2) % n, sgn);
      acc[r] = czero();
    }
    for (int p1 = n1 - 1; p1 >= 0; --p1) {
      cplx v = x[(p1 * n2 + p2) * stride];
#pragma unroll
      for (int r = 0; r < Q; ++r) acc[r] = cadd(cmul(acc[r], z[r]), v);
    }
#pragma unroll
    for (int r = 0; r < Q; ++r) {
      int q1 = g * Q + r;
      if (q1 < n1) t[(q1 * n2 + p2) * stride] = cmul(acc[r], root(tw, (p2 * q1) % n, sgn));
    }
  }
  __syncthreads();
  // stage B: item = (array, line, q1, group of 8 q2)
  const int groups = (n2 + Q - 1) / Q;
  int itemsB = 2 * nlines * n1 * groups;
  for (int it = threadIdx.x; it < itemsB; it += blockDim.x) {
    int arr = it / (nlines * n1 * groups);
    int rem = it - arr * nlines * n1 * groups;
    int line = rem / (n1 * groups);
    rem -= line * n1 * groups;
    int q1 = rem / groups, g = rem - (rem / groups) * groups;
    const cplx* t = (arr ? t1 : t0) + line * line_mul + q1 * n2 * stride;
    cplx* x = (arr ? x1 : x0) + line * line_mul;
    cplx z[Q], acc[Q];
#pragma unroll
    for (int r = 0; r < Q; ++r) {
      int q2 = g * Q + r;
      z[r] = root(tw, ((q2 < n2 ? q2 : 0) * n1) % n, sgn);
      acc[r] = czero();
    }
    for (int p2 = n2 - 1; p2 >= 0; --p2) {
      cplx v = t[p2 * stride];
#pragma unroll
      for (int r = 0; r < Q; ++r) acc[r] = cadd(cmul(acc[r], z[r]), v);
    }
#pragma unroll
    for (int r = 0; r < Q; ++r) {
      int q2 = g * Q + r;
      if (q2 < n2) x[(q1 + n1 * q2) * stride] = cscal(acc[r], scale);
    }
  }
  __syncthreads();
}

// fft_split for sizes known at compile time
constexpr int fft_split_ct(int n) {
  int best = 1;
  for (int f = 2; f * f <= n; ++f)
    if (n % f == 0) best = f;
  return best;
}

// axis_dft with the line length, line count and layout fixed at compile time: the same two
// Cooley-Tukey stages, with every loop unrolled so that the Horner chains of different outputs
// are independent instruction streams (composite n only).
template <int N, int NLINES, int LM, int ST>
__device__ __forceinline__ void axis_dft_ct(cplx* __restrict__ x0, cplx* __restrict__ x1, cplx* __restrict__ t0,
                                            cplx* __restrict__ t1, const cplx* __restrict__ tw, int sgn, double scale) {
  constexpr int N1 = fft_split_ct(N), N2 = N / N1;
  static_assert(N1 > 1, "prime line lengths take the runtime transform");
  constexpr int IA = 2 * NLINES * N2;  // stage A items: (array, line, p2)
#pragma unroll
  for (int it0 = 0; it0 < IA; it0 += 256) {
    int it = it0 + threadIdx.x;
    if (it < IA) {
      int arr = it / (NLINES * N2);
      int rem = it - arr * NLINES * N2;
      int line = rem / N2, p2 = rem - (rem / N2) * N2;
      const cplx* x = (arr ? x1 : x0) + line * LM;
      cplx* t = (arr ? t1 : t0) + line * LM;
      cplx v[N1];
#pragma unroll
      for (int p1 = 0; p1 < N1; ++p1) v[p1] = x[(p1 * N2 + p2) * ST];
#pragma unroll
      for (int q1 = 0; q1 < N1; ++q1) {
        cplx r = root(tw, (N2 * q1) % N, sgn), acc = czero();
#pragma unroll
        for (int p1 = N1 - 1; p1 >= 0; --p1) acc = cadd(cmul(acc, r), v[p1]);
        t[(q1 * N2 + p2) * ST] = cmul(acc, root(tw, (p2 * q1) % N, sgn));
      }
    }
  }
  __syncthreads();
  constexpr int IB = 2 * NLINES * N1;  // stage B items: (array, line, q1), all N2 outputs each
#pragma unroll
  for (int it0 = 0; it0 < IB; it0 += 256) {
    int it = it0 + threadIdx.x;
    if (it < IB) {
      int arr = it / (NLINES * N1);
      int rem = it - arr * NLINES * N1;
      int line = rem / N1, q1 = rem - (rem / N1) * N1;
      const cplx* t = (arr ? t1 : t0) + line * LM + q1 * N2 * ST;
      cplx* x = (arr ? x1 : x0) + line * LM;
      cplx z[N2], acc[N2];
#pragma unroll
      for (int q2 = 0; q2 < N2; ++q2) {
        z[q2] = root(tw, (q2 * N1) % N, sgn);
        acc[q2] = czero();
      }
#pragma unroll
      for (int p2 = N2 - 1; p2 >= 0; --p2) {
        cplx v = t[p2 * ST];
#pragma unroll
        for (int q2 = 0; q2 < N2; ++q2) acc[q2] = cadd(cmul(acc[q2], z[q2]), v);
      }
#pragma unroll
      for (int q2 = 0; q2 < N2; ++q2) x[(q1 + N1 * q2) * ST] = cscal(acc[q2], scale);
    }
  }
  __syncthreads();
}

// Power-of-two line length n (one line per array, contiguous): Stockham autosort FFT in
// radix-4 stages (one radix-2 stage first when log2 n is odd), ping-ponging between x and the
// scratch t. Stage with sub-length Ns (the product of the radices before it) and radix R:
// butterfly j reads x[j + r n/R], r < R, multiplies by w^{sgn (j mod Ns) r n/(Ns R)}, takes the
// R-point transform and writes y[(j / Ns) Ns R + (j mod Ns) + r Ns]; after the last stage the
// output is in natural order (n log4 n work instead of n (n1 + n2)). The scale is applied by
// the last stage; a result left in the scratch is copied back. Roots from the LDS table tw
// (n entries). Every stage ends with a block barrier; the caller synchronises before the first.
__device__ __forceinline__ void axis_fft_pow2(cplx* __restrict__ x0, cplx* __restrict__ x1, cplx* __restrict__ t0,
                                              cplx* __restrict__ t1, int n, const cplx* __restrict__ tw, int sgn,
                                              double scale) {
  int lg = 0;
  while ((1 << lg) < n) ++lg;
  cplx *s0 = x0, *s1 = x1, *d0 = t0, *d1 = t1;
  // Ns, R and n are powers of two: the index arithmetic below is shifts and masks
  int lgNs = 0;
  int rem = lg;
  while (rem > 0) {
    const int lgR = (rem & 1) ? 1 : 2;  // the radix-2 stage first, then radix 4
    const int R = 1 << lgR, Ns = 1 << lgNs;
    rem -= lgR;
    const bool last = rem == 0;
    const double sc = last ? scale : 1.0;
    const int nb = n >> lgR;                // butterflies per array
    const int lgu = lg - lgNs - lgR;        // root step of a butterfly: n / (Ns R) per unit of j mod Ns
    for (int it = threadIdx.x; it < 2 * nb; it += blockDim.x) {
      const int arr = it >= nb;
      const int j = it - arr * nb;
      const cplx* src = arr ? s1 : s0;
      cplx* dst = arr ? d1 : d0;
      const int jm = j & (Ns - 1);
      const int ustep = jm << lgu;
      const int base = ((j >> lgNs) << (lgNs + lgR)) + jm;
      if (R == 2) {
        cplx a = src[j], b = cmul(src[j + nb], root(tw, ustep, sgn));
        dst[base] = cscal(cadd(a, b), sc);
        dst[base + Ns] = cscal(csub(a, b), sc);
      } else {
        cplx v0 = src[j];
        cplx v1 = cmul(src[j + nb], root(tw, ustep, sgn));
        cplx v2 = cmul(src[j + 2 * nb], root(tw, (2 * ustep) & (n - 1), sgn));
        cplx v3 = cmul(src[j + 3 * nb], root(tw, (3 * ustep) & (n - 1), sgn));
        cplx s02 = cadd(v0, v2), d02 = csub(v0, v2), s13 = cadd(v1, v3), d13 = csub(v1, v3);
        cplx id13 = sgn > 0 ? cmuli(d13) : cneg(cmuli(d13));  // (sgn i) (v1 - v3)
        dst[base] = cscal(cadd(s02, s13), sc);
        dst[base + Ns] = cscal(cadd(d02, id13), sc);
        dst[base + 2 * Ns] = cscal(csub(s02, s13), sc);
        dst[base + 3 * Ns] = cscal(csub(d02, id13), sc);
      }
    }
    __syncthreads();
    lgNs += lgR;
    cplx* q0 = s0;
    cplx* q1 = s1;
    s0 = d0;
    s1 = d1;
    d0 = q0;
    d1 = q1;
  }
  if (s0 != x0) {  // an odd number of stages left the result in the scratch
    for (int it = threadIdx.x; it < 2 * n; it += blockDim.x) {
      if (it < n) x0[it] = t0[it];
      else x1[it - n] = t1[it - n];
    }
    __syncthreads();
  }
}

// Index transform of an nx x ny grid (k = ix * ny + iy) for two arrays in place:
//   x(R) <- scale * sum_k e^{sgn 2 pi i (ix Rx / nx + iy Ry / ny)} x(k); y lines, then x lines.
__device__ __forceinline__ void grid_dft(cplx* x0, cplx* x1, cplx* t0, cplx* t1, int nx, int ny, const cplx* twx,
                                         const cplx* twy, int sgn, double scale) {
  if (ny == 1 && nx >= 128 && (nx & (nx - 1)) == 0) {  // long power-of-two chains
    axis_fft_pow2(x0, x1, t0, t1, nx, twx, sgn, scale);
    return;
  }
  if (ny > 1) axis_dft(x0, x1, t0, t1, ny, nx, ny, 1, twy, sgn, 1.0);
  axis_dft(x0, x1, t0, t1, nx, ny, 1, ny, twx, sgn, scale);
}
// grid_dft for grid sizes fixed at compile time (NY = 1: a chain, only the x lines)
template <int NX, int NY>
__device__ __forceinline__ void grid_dft_ct(cplx* x0, cplx* x1, cplx* t0, cplx* t1, const cplx* twx, const cplx* twy,
                                            int sgn, double scale) {
  if constexpr (NY > 1) axis_dft_ct<NY, NX, NY, 1>(x0, x1, t0, t1, twy, sgn, 1.0);
  axis_dft_ct<NX, NY, 1, NY>(x0, x1, t0, t1, twx, sgn, scale);
}

}  // namespace kbe
