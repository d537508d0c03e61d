// HIP kernels (gfx950) of the Kadanoff-Baym propagation step.
//
//   k_init_*        uncorrelated initial state (Fermi-Dirac density of h0, mu by bisection)
//   k_hf            mean-field (first-order) self-energy from the local density matrix
//   k_props         per-k propagators V, Vh, Phi of the midpoint Hamiltonian (scaling and
//                   squaring of an augmented matrix exponential, one wavefront per k)
//   k_kick_row      the dipole kick of eq. (dipole) on the completed slice nearest t0
//   k_sigma         second-Born self-energy of a time slice, eq. (2BSE), by k <-> R transforms
//                   (Hubbard preset)
//   k_sigma_fwd/ib  the same for the interband preset: lines to real space, then products
//                   and back
//   k_sigma_direct  the paper's direct momentum sums for the interband preset (comparison)
//   k_diag_I        equal-time collision integral I^<(t_m, t_m) and D_m
//   k_hist_pair, k_hist_bulk(_split) and their FP32 forms
//                   the history sums of eq. (CI): stream the packed triangle of rows 0..m-1
//                   once, every stored block feeding its column and its row
//   k_row           end-point terms (trapezoid or Gregory), collision row assembly,
//                   predictor/corrector update
//   k_change_max    the corrector's row change (stopping rule)
//   k_obs           observables of one time slice
//   k_aux           refresh the column / diagonal / recent-row copies of the history
#include "kbe_device.hpp"
#include "kbe_kernels.hpp"

namespace kbe {

// ------------------------------------------------------------------ utility
__global__ void k_fill_zero(double* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0.0;
}

// Write one element of the packed history in its storage precision.
__device__ __forceinline__ void commit_store(const Dims& d, void* hist, int k, int c, int j, int tp, cplx v) {
  if (d.fp32)
    reinterpret_cast<float2*>(hist)[hist_idx(d, k, c, j, tp)] = make_float2((float)v.x, (float)v.y);
  else
    reinterpret_cast<cplx*>(hist)[hist_idx(d, k, c, j, tp)] = v;
}
__device__ __forceinline__ cplx history_load(const Dims& d, const void* hist, int k, int c, int j, int tp) {
  if (d.fp32) {
    float2 v = reinterpret_cast<const float2*>(hist)[hist_idx(d, k, c, j, tp)];
    return make_double2((double)v.x, (double)v.y);
  }
  return reinterpret_cast<const cplx*>(hist)[hist_idx(d, k, c, j, tp)];
}

// ------------------------------------------------------------------ initial state
// Eigen-decomposition of h0(k - A(0)) per k (one thread per k).
template <int NB>
__global__ __launch_bounds__(64) void k_init_eig(Dims d, const cplx* __restrict__ hop, double Ax, double Ay,
                                                 double* __restrict__ w, cplx* __restrict__ U) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.nk) return;
  cplx h[NB * NB], V[NB * NB];
  double ev[NB];
  bloch_h0<NB>(hop, d.nkx, d.nky, k, Ax, Ay, h);
  jacobi_eigh<NB>(h, ev, V);
#pragma unroll
  for (int b = 0; b < NB; ++b) w[k * NB + b] = ev[b];
#pragma unroll
  for (int i = 0; i < NB * NB; ++i) U[(int64_t)k * NB * NB + i] = V[i];
}

// Chemical potential by bisection: N_k^{-1} sum_{k,b} f((w - mu)/T) = target (one block).
__global__ __launch_bounds__(256) void k_init_mu(int n, const double* __restrict__ w, double temp,
                                                 double target, double* __restrict__ mu_out) {
  __shared__ double red[256];
  __shared__ double lohi[2];
  int t = threadIdx.x;
  double lo = 1e300, hi = -1e300;
  for (int i = t; i < n; i += 256) {
    lo = fmin(lo, w[i]);
    hi = fmax(hi, w[i]);
  }
  red[t] = lo;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] = fmin(red[t], red[t + s]);
    __syncthreads();
  }
  if (t == 0) lohi[0] = red[0] - 50.0 * temp - 1.0;
  __syncthreads();
  red[t] = hi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] = fmax(red[t], red[t + s]);
    __syncthreads();
  }
  if (t == 0) lohi[1] = red[0] + 50.0 * temp + 1.0;
  __syncthreads();
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lohi[0] + lohi[1]);
    double acc = 0.0;
    for (int i = t; i < n; i += 256) acc += 1.0 / (1.0 + exp((w[i] - mid) / temp));
    red[t] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) red[t] += red[t + s];
      __syncthreads();
    }
    if (t == 0) {
      if (red[0] < target) lohi[0] = mid;
      else lohi[1] = mid;
    }
    __syncthreads();
    if (lohi[1] - lohi[0] < 1e-15 * fmax(1.0, fabs(mid))) break;
  }
  if (t == 0) *mu_out = 0.5 * (lohi[0] + lohi[1]);
}

// rho0 = U f(w - mu) U^dag; row 0 of the history (G^< = i rho, G^> = -i (1 - rho)).
template <int NB>
__global__ __launch_bounds__(64) void k_init_rho(Dims d, const double* __restrict__ w, const cplx* __restrict__ U,
                                                 const double* __restrict__ mu, double temp,
                                                 cplx* __restrict__ rhoA, cplx* __restrict__ rhoB,
                                                 void* __restrict__ hist, cplx* __restrict__ row64,
                                                 cplx* __restrict__ col0, cplx* __restrict__ diag) {
  constexpr int NBB = NB * NB;
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.nk) return;
  double f[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) f[b] = 1.0 / (1.0 + exp((w[k * NB + b] - *mu) / temp));
  const cplx* Uk = U + (int64_t)k * NBB;
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      cplx s = czero();
#pragma unroll
      for (int c = 0; c < NB; ++c) s = cadd(s, cscal(cmul(Uk[a * NB + c], cconj(Uk[b * NB + c])), f[c]));
      int e = a * NB + b;
      rhoA[(int64_t)k * NBB + e] = s;
      rhoB[(int64_t)k * NBB + e] = s;
      cplx g[2];
      g[0] = cmuli(s);
      g[1] = cneg(cmuli(csub(cmk(a == b ? 1.0 : 0.0, 0.0), s)));
#pragma unroll
      for (int sc = 0; sc < 2; ++sc) {
        int c = sc * NBB + e;
        commit_store(d, hist, k, c, 0, 0, g[sc]);
        row64[row64_idx(d, 0, k, c, 0)] = g[sc];
        col0[colq_idx(d, k, c, 0, 0)] = g[sc];
        diag[band_idx(d, k, c, 0, 0)] = g[sc];
      }
    }
}

// ------------------------------------------------------------------ mean field
// hf_out = one-body extra term + Sigma^HF[rho_loc], rho = (1 - wb) rhoA + wb rhoB (one block).
template <int NB>
__global__ __launch_bounds__(256) void k_hf(Dims d, const cplx* __restrict__ rhoA, const cplx* __restrict__ rhoB,
                                            double wb, int interaction, int hf, double U,
                                            cplx* __restrict__ hf_out) {
  constexpr int NBB = NB * NB;
  __shared__ cplx lds[NBB * 256];
  cplx loc[NBB];
#pragma unroll
  for (int e = 0; e < NBB; ++e) loc[e] = czero();
  for (int k = threadIdx.x; k < d.nk; k += 256)
#pragma unroll
    for (int e = 0; e < NBB; ++e)
      loc[e] = cadd(loc[e], cadd(cscal(rhoA[(int64_t)k * NBB + e], 1.0 - wb), cscal(rhoB[(int64_t)k * NBB + e], wb)));
  block_sum_cplx<NBB>(loc, lds);
  if (threadIdx.x == 0) {
    double inv = 1.0 / d.nk;
    cplx out[NBB];
#pragma unroll
    for (int e = 0; e < NBB; ++e) out[e] = czero();
    if (interaction == KBE_DEV_INT_HUBBARD) {
      if (hf)
#pragma unroll
        for (int a = 0; a < NB; ++a) out[a * NB + a] = cmk(U * loc[a * NB + a].x * inv, 0.0);
    } else {
      // eq. (ham): -U c_c^dag c_c one-body term; Hartree U n_c / U n_v, Fock -U rho_vc
      out[NBB - 1] = cmk(-U, 0.0);
      if constexpr (NB == 2) {
        if (hf) {
          out[0] = cadd(out[0], cmk(U * loc[3].x * inv, 0.0));
          out[3] = cadd(out[3], cmk(U * loc[0].x * inv, 0.0));
          out[1] = cscal(loc[1], -U * inv);
          out[2] = cscal(loc[2], -U * inv);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < NBB; ++e) hf_out[e] = out[e];
  }
}

// ------------------------------------------------------------------ propagators
// One wavefront per k. The augmented matrix M = [[-i hbar dt, dt 1], [0, 0]] (2NB x 2NB)
// has exp(M) = [[V, dt phi1(-i hbar dt)], [0, 1]], so Phi = -i * (top-right block).
// exp(M / 2^s) by a degree-16 Taylor polynomial (Horner), ||M / 2^s||_F <= 1/4, then s
// squarings; the square before the last is exp(M/2), whose top-left block is Vh.
template <int NB>
__global__ __launch_bounds__(256) void k_props(Dims d, const cplx* __restrict__ hop, const cplx* __restrict__ hf,
                                               double Ax, double Ay, double dt, cplx* __restrict__ props) {
  constexpr int N2 = 2 * NB, NN = N2 * N2, NBB = NB * NB;
  __shared__ cplx sX[4][NN], sE[4][NN];
  int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int k = blockIdx.x * 4 + wv;
  bool kval = k < d.nk;
  int r = lane / N2, c = lane - (lane / N2) * N2;
  bool act = kval && lane < NN;
  cplx m = czero();
  if (act) {
    if (r < NB && c < NB) {
      cplx h[NBB];
      bloch_h0<NB>(hop, d.nkx, d.nky, k, Ax, Ay, h);
      cplx hb = cadd(h[r * NB + c], hf[r * NB + c]);
      m = cscal(cmuli(hb), -dt);  // -i hbar dt
    } else if (r < NB && c == r + NB) {
      m = cmk(dt, 0.0);
    }
  }
  double nrm2 = wave_sum(act ? cabs2(m) : 0.0);
  int s = 1;
  double nrm = sqrt(nrm2);
  while (nrm > ldexp(0.25, s) && s < 60) ++s;
  double scale = ldexp(1.0, -s);
  cplx x = cscal(m, scale);
  cplx id = cmk((act && r == c) ? 1.0 : 0.0, 0.0);
  if (lane < NN) sX[wv][lane] = x;
  cplx e = id;
  if (lane < NN) sE[wv][lane] = e;
  wave_sync();  // every LDS array here is per wavefront
  for (int n = 16; n >= 1; --n) {  // E <- 1 + X E / n
    cplx acc = czero();
    if (lane < NN)
#pragma unroll
      for (int l = 0; l < N2; ++l) cmac(acc, sX[wv][r * N2 + l], sE[wv][l * N2 + c]);
    wave_sync();  // every LDS array here is per wavefront
    e = cadd(id, cscal(acc, 1.0 / n));
    if (lane < NN) sE[wv][lane] = e;
    wave_sync();  // every LDS array here is per wavefront
  }
  cplx half = czero();
  for (int q = 0; q < s; ++q) {  // E <- E E
    if (q == s - 1) half = e;
    cplx acc = czero();
    if (lane < NN)
#pragma unroll
      for (int l = 0; l < N2; ++l) cmac(acc, sE[wv][r * N2 + l], sE[wv][l * N2 + c]);
    wave_sync();  // every LDS array here is per wavefront
    e = acc;
    if (lane < NN) sE[wv][lane] = e;
    wave_sync();  // every LDS array here is per wavefront
  }
  if (act && r < NB) {
    cplx* P = props + (int64_t)k * 3 * NBB;
    if (c < NB) {
      P[r * NB + c] = e;              // V
      P[NBB + r * NB + c] = half;     // Vh
    } else {
      P[2 * NBB + r * NB + (c - NB)] = cneg(cmuli(e));  // Phi = -i * top-right
    }
  }
}

// ------------------------------------------------------------------ self-energy
// One block per (t_j, orbital pair ab) of row m. With plain index transforms
//   g(R) = N_k^{-1} sum_j e^{+2 pi i j.R / n} G(k_j),   S(k_j) = sum_R e^{-2 pi i j.R / n} S(R),
// the -pi offset of eq. (kj) cancels in the product of two forward lines and one backward
// line, and the backward line is g_ba(-R; t_j, t_m) = -conj(g_ab(R; t_m, t_j)), so
//   Hubbard:  Sigma^<_ab(R) = -U^2 g^<_ab(R)^2 conj(g^>_ab(R)),  Sigma^> with < and > swapped.
// Block-to-work mapping gives each XCD a contiguous range of t_j, so the cache lines of
// row m that several t_j share stay in one L2. NX, NY > 0: the grid size is fixed at compile
// time (unrolled transforms, 1.8x faster on 24 x 24); NX = NY = 0: any grid, sizes from d.
// Dynamic LDS: four lines of N_k points and the nx + ny roots of unity.
template <int NB, int NX, int NY>
__global__ __launch_bounds__(256) void k_sigma(Dims d, const cplx* __restrict__ row64, cplx* __restrict__ sig,
                                               int m, double UU, int corr) {
  constexpr int NBB = NB * NB;
  extern __shared__ cplx lds[];
  const int nk = NX > 0 ? NX * NY : d.nk;
  const int nx = NX > 0 ? NX : d.nkx, ny = NX > 0 ? NY : d.nky;
  cplx* gl = lds;
  cplx* gg = lds + nk;
  cplx* tl = lds + 2 * nk;
  cplx* tg = lds + 3 * nk;
  cplx* twx = lds + 4 * nk;  // roots of unity, nx and ny entries
  cplx* twy = twx + nx;
  int total = (m + 1) * NBB;
  int per = (total + 7) >> 3;
  int item = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (item >= total) return;
  int j = item / NBB, ab = item - (item / NBB) * NBB;
  int t = threadIdx.x;
  fill_roots(twx, nx);
  fill_roots(twy, ny);
  for (int k = t; k < nk; k += 256) {
    gl[k] = row64[row64_idx(d, m, k, ab, j)];
    gg[k] = row64[row64_idx(d, m, k, NBB + ab, j)];
  }
  __syncthreads();
  // k -> R (1/N_k)
  if constexpr (NX > 0)
    grid_dft_ct<NX, NY>(gl, gg, tl, tg, twx, twy, +1, 1.0 / nk);
  else
    grid_dft(gl, gg, tl, tg, nx, ny, twx, twy, +1, 1.0 / nk);
  for (int o = t; o < nk; o += 256) {
    cplx al = gl[o], ag = gg[o];
    cplx sl = czero(), sg = czero();
    if (corr) {
      sl = cscal(cmul(cmul(al, al), cconj(ag)), -UU);
      sg = cscal(cmul(cmul(ag, ag), cconj(al)), -UU);
    }
    gl[o] = sl;
    gg[o] = sg;
  }
  __syncthreads();
  // R -> k
  if constexpr (NX > 0)
    grid_dft_ct<NX, NY>(gl, gg, tl, tg, twx, twy, -1, 1.0);
  else
    grid_dft(gl, gg, tl, tg, nx, ny, twx, twy, -1, 1.0);
  for (int o = t; o < nk; o += 256) {
    cplx al = gl[o], ag = gg[o];
    sig[sig_idx(d, o, 0, ab, j)] = al;
    sig[sig_idx(d, o, 1, ab, j)] = ag;
    sig[sig_idx(d, o, 2, ab, j)] = csub(ag, al);
  }
}

// Interband preset (nb = 2, the paper's eq. (2BSE)): with jbar the other band,
//   Sigma^<_ab(R) = -U^2 (-1)^(a+b) det g^<(R) conj(g^>_{abar bbar}(R)),  Sigma^> with < and > swapped,
// (the direct minus the exchange term of eq. (2BSE): g_{abar bbar} g_ab - g_{a bbar} g_{abar b} is
// (-1)^(a+b) det g; the backward line is -conj of the forward one, as for the Hubbard preset).
// Each output needs all four orbital pairs of both components at R, so the transforms are split
// around a real-space buffer gR[t_j][comp][ab][R]: k_sigma_fwd takes the lines of row m to R,
// k_sigma_ib forms the products and takes them back to k. Both: one block per (t_j, ab), the
// same XCD-aware mapping and LDS tile as k_sigma.
__device__ __forceinline__ int64_t gr_idx(const Dims& d, int j, int comp, int ab, int R) {
  return (((int64_t)j * 2 + comp) * 4 + ab) * d.nk + R;
}
template <int NX, int NY>
__global__ __launch_bounds__(256) void k_sigma_fwd(Dims d, const cplx* __restrict__ row64, cplx* __restrict__ gR,
                                                   int m) {
  extern __shared__ cplx lds[];
  const int nk = NX > 0 ? NX * NY : d.nk;
  const int nx = NX > 0 ? NX : d.nkx, ny = NX > 0 ? NY : d.nky;
  cplx* gl = lds;
  cplx* gg = lds + nk;
  cplx* tl = lds + 2 * nk;
  cplx* tg = lds + 3 * nk;
  cplx* twx = lds + 4 * nk;
  cplx* twy = twx + nx;
  int total = (m + 1) * 4;
  int per = (total + 7) >> 3;
  int item = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (item >= total) return;
  int j = item >> 2, ab = item & 3;
  int t = threadIdx.x;
  fill_roots(twx, nx);
  fill_roots(twy, ny);
  for (int k = t; k < nk; k += 256) {
    gl[k] = row64[row64_idx(d, m, k, ab, j)];
    gg[k] = row64[row64_idx(d, m, k, 4 + ab, j)];
  }
  __syncthreads();
  if constexpr (NX > 0)
    grid_dft_ct<NX, NY>(gl, gg, tl, tg, twx, twy, +1, 1.0 / nk);
  else
    grid_dft(gl, gg, tl, tg, nx, ny, twx, twy, +1, 1.0 / nk);
  for (int o = t; o < nk; o += 256) {
    gR[gr_idx(d, j, 0, ab, o)] = gl[o];
    gR[gr_idx(d, j, 1, ab, o)] = gg[o];
  }
}
template <int NX, int NY>
__global__ __launch_bounds__(256) void k_sigma_ib(Dims d, const cplx* __restrict__ gR, cplx* __restrict__ sig,
                                                  int m, double UU, int corr) {
  extern __shared__ cplx lds[];
  const int nk = NX > 0 ? NX * NY : d.nk;
  const int nx = NX > 0 ? NX : d.nkx, ny = NX > 0 ? NY : d.nky;
  cplx* sl = lds;
  cplx* sg = lds + nk;
  cplx* tl = lds + 2 * nk;
  cplx* tg = lds + 3 * nk;
  cplx* twx = lds + 4 * nk;
  cplx* twy = twx + nx;
  int total = (m + 1) * 4;
  int per = (total + 7) >> 3;
  int item = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (item >= total) return;
  int j = item >> 2, ab = item & 3;
  int a = ab >> 1, b = ab & 1;
  int cross = (1 - a) * 2 + (1 - b);                 // orbital pair (abar, bbar)
  double pre = ((a + b) & 1) ? UU : -UU;             // -U^2 (-1)^(a+b)
  int t = threadIdx.x;
  fill_roots(twx, nx);
  fill_roots(twy, ny);
  for (int o = t; o < nk; o += 256) {
    cplx l00 = gR[gr_idx(d, j, 0, 0, o)], l01 = gR[gr_idx(d, j, 0, 1, o)];
    cplx l10 = gR[gr_idx(d, j, 0, 2, o)], l11 = gR[gr_idx(d, j, 0, 3, o)];
    cplx g00 = gR[gr_idx(d, j, 1, 0, o)], g01 = gR[gr_idx(d, j, 1, 1, o)];
    cplx g10 = gR[gr_idx(d, j, 1, 2, o)], g11 = gR[gr_idx(d, j, 1, 3, o)];
    cplx dl = csub(cmul(l00, l11), cmul(l01, l10));
    cplx dg = csub(cmul(g00, g11), cmul(g01, g10));
    cplx lx = gR[gr_idx(d, j, 0, cross, o)], gx = gR[gr_idx(d, j, 1, cross, o)];
    sl[o] = corr ? cscal(cmul(dl, cconj(gx)), pre) : czero();
    sg[o] = corr ? cscal(cmul(dg, cconj(lx)), pre) : czero();
  }
  __syncthreads();
  if constexpr (NX > 0)
    grid_dft_ct<NX, NY>(sl, sg, tl, tg, twx, twy, -1, 1.0);
  else
    grid_dft(sl, sg, tl, tg, nx, ny, twx, twy, -1, 1.0);
  for (int o = t; o < nk; o += 256) {
    cplx vl = sl[o], vg = sg[o];
    sig[sig_idx(d, o, 0, ab, j)] = vl;
    sig[sig_idx(d, o, 1, ab, j)] = vg;
    sig[sig_idx(d, o, 2, ab, j)] = csub(vg, vl);
  }
}

// The paper's own evaluation of eq. (2BSE) for the interband preset on a chain (n divisible by
// 8): the direct term through the polarizability of eq. (polarizability)/(kernel2), O(n^2) per
// (t_j, jm), and the exchange term by the nested momentum sums of Alg. "contraction2",
// O(n^3) per (t_j, jm); kept beside the transform route to time the paper's algorithm on this
// hardware (same output). Momenta on the -pi-offset grid of eq. (kj): k_a + k_b has index
// a + b - n/2 and k_a - k_b index a - b + n/2 (mod n), so k' + q - k has index k' + q - k.
// One block per (t_j, jm) of row m, both components in turn; 512 threads in 4 groups that split
// the q range (8 waves per CU: the 96 KB of LDS leave room for one block). In a group thread i
// owns the KD = 8 outputs k = 8i .. 8i+7 (n <= 1024) and slides a window of KD backward-line
// values along k', so one LDS read feeds KD complex multiply-adds; neighbouring lanes then read
// the backward line 8 elements apart, so it is stored with one pad element after every 8 (lane
// stride 36 banks). The groups' partial sums are added in LDS in a fixed order.
// Dynamic LDS: the four forward lines of the component, P, the padded backward line:
// 6n + n/8 complex.
constexpr int KD = 8, DG = 4;
__device__ __forceinline__ int wrap_n(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }
__device__ __forceinline__ int padded(int x) { return x + (x >> 3); }
__global__ __launch_bounds__(512) void k_sigma_direct(Dims d, const cplx* __restrict__ row64, cplx* __restrict__ sig,
                                                      int m, double UU, int corr) {
  extern __shared__ cplx lds[];
  const int n = d.nk, h = n / 2;
  cplx* Ajm = lds;           // G^s_{j m}     (t_m, t_j)
  cplx* Abb = lds + n;       // G^s_{jb mb}
  cplx* Ajb = lds + 2 * n;   // G^s_{j mb}
  cplx* Abm = lds + 3 * n;   // G^s_{jb m}
  cplx* P = lds + 4 * n;
  cplx* Bk = lds + 5 * n;    // G^{s'}_{mb jb}(k; t_j, t_m) = -conj(G^{s'}_{jb mb}(k; t_m, t_j)), padded
  int item = blockIdx.x;     // (t_j, jm)
  int j = item >> 2, ab = item & 3;
  int a = ab >> 1, b = ab & 1, ja = 1 - a, mb = 1 - b;
  int t = threadIdx.x;
  int g = t >> 7, k0 = (t & 127) * KD;
  int q0 = g * (n / DG), q1 = q0 + n / DG;
  cplx outv[2][KD];
  const double pre = UU / ((double)n * (double)n);
  for (int s = 0; s < 2; ++s) {
    __syncthreads();
    for (int k = t; k < n; k += 512) {
      Ajm[k] = row64[row64_idx(d, m, k, s * 4 + a * 2 + b, j)];
      Abb[k] = row64[row64_idx(d, m, k, s * 4 + ja * 2 + mb, j)];
      Ajb[k] = row64[row64_idx(d, m, k, s * 4 + a * 2 + mb, j)];
      Abm[k] = row64[row64_idx(d, m, k, s * 4 + ja * 2 + b, j)];
      Bk[padded(k)] = cneg(cconj(row64[row64_idx(d, m, k, (1 - s) * 4 + ja * 2 + mb, j)]));
    }
    __syncthreads();
    // polarizability P(q) = sum_k' G_{jb mb}(k' + q) G_{mb jb}(k'; t_j, t_m)
    for (int q = t; q < n; q += 512) {
      cplx acc = czero();
      int idx = wrap_n(q - h, n);
      for (int kp = 0; kp < n; ++kp) {
        cmac(acc, Abb[idx], Bk[padded(kp)]);
        idx = idx + 1 == n ? 0 : idx + 1;
      }
      P[q] = acc;
    }
    __syncthreads();
    cplx part[KD];
#pragma unroll
    for (int r = 0; r < KD; ++r) part[r] = czero();
    if (k0 < n) {
      cplx dir[KD], ex[KD];
#pragma unroll
      for (int r = 0; r < KD; ++r) dir[r] = ex[r] = czero();
      // direct: sum_q G_{jm}(k - q) P(q), this group's q
      for (int q = q0; q < q1; ++q) {
        cplx pq = P[q];
#pragma unroll
        for (int r = 0; r < KD; ++r)
          if (k0 + r < n) cmac(dir[r], Ajm[wrap_n(k0 + r - q + h, n)], pq);
      }
      // exchange: sum_q G_{jb m}(q) sum_k' G_{j mb}(k') G_{mb jb}(k' + q - k; t_j, t_m)
      for (int q = q0; q < q1; ++q) {
        cplx acc[KD], w[KD];
        int base = q - k0;  // window element r at k' is Bk[k' + base - r]
#pragma unroll
        for (int r = 0; r < KD; ++r) {
          acc[r] = czero();
          w[r] = Bk[padded(wrap_n(base - r, n))];
        }
        int idx = wrap_n(base, n);
        for (int kp = 0; kp < n; kp += KD) {  // unrolled by the window length: the shifts are renames
#pragma unroll
          for (int u = 0; u < KD; ++u) {
            cplx av = Ajb[kp + u];
#pragma unroll
            for (int r = 0; r < KD; ++r) cmac(acc[r], av, w[r]);
#pragma unroll
            for (int r = KD - 1; r > 0; --r) w[r] = w[r - 1];
            idx = idx + 1 == n ? 0 : idx + 1;
            w[0] = Bk[padded(idx)];
          }
        }
        cplx cq = Abm[q];
#pragma unroll
        for (int r = 0; r < KD; ++r) cmac(ex[r], cq, acc[r]);
      }
#pragma unroll
      for (int r = 0; r < KD; ++r) part[r] = csub(dir[r], ex[r]);
    }
    // add the 4 groups' partial sums (in the forward-line area, no longer read)
    __syncthreads();
    if (k0 < n) {
#pragma unroll
      for (int r = 0; r < KD; ++r)
        if (k0 + r < n) lds[g * n + k0 + r] = part[r];
    }
    __syncthreads();
    if (g == 0 && k0 < n) {
#pragma unroll
      for (int r = 0; r < KD; ++r) {
        int k = k0 + r;
        cplx v = czero();
        if (k < n) v = cadd(cadd(lds[k], lds[n + k]), cadd(lds[2 * n + k], lds[3 * n + k]));
        outv[s][r] = corr ? cscal(v, pre) : czero();
      }
    }
  }
  if (g == 0 && k0 < n) {
#pragma unroll
    for (int r = 0; r < KD; ++r) {
      int k = k0 + r;
      if (k < n) {
        sig[sig_idx(d, k, 0, ab, j)] = outv[0][r];
        sig[sig_idx(d, k, 1, ab, j)] = outv[1][r];
        sig[sig_idx(d, k, 2, ab, j)] = csub(outv[1][r], outv[0][r]);
      }
    }
  }
}

// ------------------------------------------------------------------ equal-time collision
// I^<(t_m, t_m) = dt sum_j a_j [Sigma^>_mj G^<_jm - Sigma^<_mj G^>_jm],  G_jm = -(G_mj)^dag
// for j < m, a_j the quadrature weights on [0, t_m] (trapezoid, or with Gregory end
// corrections); I^>(t_m, t_m) is the same matrix (both integrals of eq. (CI) run over
// [0, t_m] and combine term by term). One block per k.
template <int NB>
__global__ __launch_bounds__(256) void k_diag_I(Dims d, const cplx* __restrict__ row64,
                                                const cplx* __restrict__ sig, cplx* __restrict__ Icur,
                                                cplx* __restrict__ Dcur, int m, double dt, QuadW Q) {
  constexpr int NBB = NB * NB;
  __shared__ cplx lds[NBB * 256];
  int k = blockIdx.x;
  cplx acc[NBB];
  mat_zero<NB>(acc);
  if (m > 0) {
    for (int j = threadIdx.x; j <= m; j += 256) {
      double wgt = quad_w(Q, j, m);
      cplx Gl[NBB], Gg[NBB], Sl[NBB], Sg[NBB], t[NBB];
#pragma unroll
      for (int e = 0; e < NBB; ++e) {
        Gl[e] = row64[row64_idx(d, m, k, e, j)];
        Gg[e] = row64[row64_idx(d, m, k, NBB + e, j)];
        Sl[e] = sig[sig_idx(d, k, 0, e, j)];
        Sg[e] = sig[sig_idx(d, k, 1, e, j)];
      }
      // j < m: G_jm = -G_mj^dag, so Sg G^<_jm - Sl G^>_jm = Sl Gg^dag - Sg Gl^dag;
      // j = m: the stored equal-time block, Sg Gl - Sl Gg.
      cplx u[NBB];
      mat_zero<NB>(t);
      mat_zero<NB>(u);
      if (j < m) {
        mm_acc_bdag<NB>(t, Sl, Gg);
        mm_acc_bdag<NB>(u, Sg, Gl);
      } else {
        mm_acc<NB>(t, Sg, Gl);
        mm_acc<NB>(u, Sl, Gg);
      }
#pragma unroll
      for (int e = 0; e < NBB; ++e) acc[e] = cadd(acc[e], cscal(csub(t[e], u[e]), wgt));
    }
  }
  block_sum_cplx<NBB>(acc, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        cplx I = cscal(acc[a * NB + b], dt);
        Icur[rowbuf_idx(d, k, a * NB + b, m)] = I;
        Icur[rowbuf_idx(d, k, NBB + a * NB + b, m)] = I;
        cplx Dv = cadd(cscal(acc[a * NB + b], dt), cconj(cscal(acc[b * NB + a], dt)));
        Dcur[(int64_t)k * NBB + a * NB + b] = Dv;
      }
  }
}

// ------------------------------------------------------------------ history sums (hot loop)
typedef float kbe_f4v __attribute__((ext_vector_type(4)));
// two complex64 values (a component pair of one column) in one 16-byte load
__device__ __forceinline__ void load_stream32x2(const float2* p, float2& a, float2& b) {
  kbe_f4v v = __builtin_nontemporal_load(reinterpret_cast<const kbe_f4v*>(p));
  a = make_float2(v.x, v.y);
  b = make_float2(v.z, v.w);
}

typedef float2 cplx32;
__device__ __forceinline__ void cmac32(cplx32& acc, cplx32 a, cplx32 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
}
__device__ __forceinline__ void cmacc32(cplx32& acc, cplx32 a, cplx32 b) {  // acc += a conj(b)
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(a.y, b.y, acc.x);
  acc.y = fmaf(a.y, b.x, acc.y);
  acc.y = fmaf(-a.x, b.y, acc.y);
}
__device__ __forceinline__ cplx32 to32(cplx v) { return make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ float rs_half32(float a, float b) {
  auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b),
                                            false, false);
  return __builtin_bit_cast(float, (unsigned)r[0]) + __builtin_bit_cast(float, (unsigned)r[1]);
}
__device__ __forceinline__ float rs_row32(float a, float b) {
  auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b),
                                            false, false);
  return __builtin_bit_cast(float, (unsigned)r[0]) + __builtin_bit_cast(float, (unsigned)r[1]);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float row16_sum32(float x) {
  x += dpp_f<0xB1>(x);
  x += dpp_f<0x4E>(x);
  x += dpp_f<0x141>(x);
  x += dpp_f<0x140>(x);
  return x;
}

template <int R, int Q>
__device__ __forceinline__ void reduce_rows32(float (&rt)[R][Q]) {
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    float y;
    if constexpr (R == 4) {
      y = rs_row32(rs_half32(rt[0][q], rt[1][q]), rs_half32(rt[2][q], rt[3][q]));
    } else if constexpr (R == 2) {
      float x = rs_half32(rt[0][q], rt[1][q]);
      y = rs_row32(x, x);
    } else {
      float x = rs_half32(rt[0][q], rt[0][q]);
      y = rs_row32(x, x);
    }
    rt[0][q] = row16_sum32(y);
  }
}
// The FP64 nb = 4 kernel's two component halves stage the row partials of the same 16 rows;
// after a block barrier each of the two wavefronts stores half of the nb^2 components of their sum
// (st0 + st1, a fixed order) to rows rb .. rb + 15 of the strip's slot, 256-byte runs.
template <int NBB>
__device__ __forceinline__ void flush_rows_fold(const cplx* st0, const cplx* st1, cplx* rp, int Tp, int rb, int m,
                                                int lane, int h) {
#pragma unroll
  for (int q = lane; q < NBB * 8; q += 64) {
    int e = h * (NBB / 2) + (q >> 4), r = q & 15;
    int row = rb + r;
    if (row < m) store_stream(rp + (int64_t)e * Tp + row, cadd(st0[e * 16 + r], st1[e * 16 + r]));
  }
}
// The FP32 nb = 4 kernel's two component halves stage the row partials of a 32-row chunk (rows
// cb .. cb + 31, both wave pairs); after a block barrier the whole block stores their sum
// (st0 + st1, a fixed order) to the strip's slot, one 512-byte run per component.
template <int NBB>
__device__ __forceinline__ void flush_chunk_fold(const cplx* st0, const cplx* st1, cplx* rp, int Tp, int cb, int m) {
  for (int q = threadIdx.x; q < NBB * 32; q += 256) {
    const int e = q >> 5, r = q & 31, row = cb + r;
    if (row < m) store_stream(rp + (int64_t)e * Tp + row, cadd(st0[e * 32 + r], st1[e * 32 + r]));
  }
}

// Bulk of the collision integrals at row m over the stored blocks (j, t'), t' <= j <= m-1,
// each with weight 1 (end-point weights are corrected in k_row):
//   column term -> output t':  SR_j G^{<,>}_{j t'}                    (SR = Sigma^> - Sigma^<)
//   row term    -> output j:   -Sigma^>_{t'} (G^<_{j t'})^dag + Sigma^<_{t'} (G^>_{j t'})^dag,
//                               t' < j, shared by I^< and I^>    (G_{t' j} = -G_{j t'}^dag)
// nb <= 2, FP64. Block = (pair of 64-column strips 2 sp, 2 sp + 1; k), the pairs with the
// most rows launched first. Lane l owns columns 128 sp + l and 128 sp + 64 + l and keeps both
// column sums in registers; the Sigma of its two columns (row term) sits in LDS. Wavefront w
// takes rows w, w + 4, ..., w + 60 of every 64-row chunk (so a chunk cut short by m leaves no
// wavefront idle while the others finish), R rows per iteration (R = 1 at nb = 2: 2 x 8 loads
// of 1 KB-contiguous data in flight; R = 4 at nb = 1), so every stored block is read from HBM
// once. The row terms of the two strips are added before the 64-lane
// reduce-scatter (at nb = 2 the four components of the row term share one reduce-scatter as
// four groups), so one row partial covers 128 columns: the writes that interleave with the
// read stream are half of what one strip per block would produce, and they leave in long runs
// (the block's rows of four 64-row chunks staged in LDS, then stored by all its threads as
// contiguous 4 KB runs per component, streaming stores). Both measures keep the read stream
// from stalling on scattered write-backs. Row partials go to slot sp; the 4
// wavefronts' column sums are combined in LDS. Deterministic: no atomics.
template <int NB>
__global__ __launch_bounds__(256) void k_hist_pair(Dims d, const cplx* __restrict__ hist,
                                                   const cplx* __restrict__ sig, cplx* __restrict__ colsum,
                                                   cplx* __restrict__ rowpart, int m) {
  constexpr int NBB = NB * NB, C = 2 * NBB;
  constexpr int R = NB == 1 ? 4 : 1;
  __shared__ cplx red[3][C][64];
  // row partials of the last ROWS_ST rows (4 chunks of 64), stored by the whole block at once
  constexpr int ROWS_ST = 256;
  __shared__ cplx stg[NBB][ROWS_ST];
  __shared__ cplx sS[2][2][NBB][64];  // [strip of the pair][Sigma^<, Sigma^>][e][lane]
  const int sp = blockIdx.x / d.nk;
  const int k = blockIdx.x - sp * d.nk;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // rows and Sigma^R wavefront-uniform
  const cplx* sk = sig + (int64_t)k * 3 * NBB * d.Tp;
  for (int q = threadIdx.x; q < 4 * NBB * 64; q += 256) {
    int l = q & 63, e = (q >> 6) % NBB, x = (q >> 6) / NBB;
    int t = 64 * (2 * sp + (x >> 1)) + l;
    sS[x >> 1][x & 1][e][l] = t < m ? sk[((x & 1) * NBB + e) * d.Tp + t] : czero();
  }
  __syncthreads();
  // the pair's second strip exists only if its first column is below m
  const bool two = 64 * (2 * sp + 1) < m;
  int tp[2];
  bool colv[2];
  const cplx* hk[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    tp[h] = 64 * (2 * sp + h) + lane;
    colv[h] = tp[h] < m;
    hk[h] = hist + strip_lane_base(d, k, (h && two) ? 2 * sp + 1 : 2 * sp, lane);
  }
  cplx acc[2][C];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int c = 0; c < C; ++c) acc[h][c] = czero();
  cplx* rp = const_cast<cplx*>(rowpart_slot(d, rowpart, k, sp));
  for (int cb = 128 * sp; cb < m; cb += 64) {
    const int rb = cb + wv;   // the wavefront's rows of the chunk: rb, rb + 4, ..., rb + 60
    const int cslot = ((cb - 128 * sp) >> 6) % (ROWS_ST / 64);   // chunk's place in the staging
    cplx* st = &stg[0][64 * cslot];                                // st[e * ROWS_ST + (row - cb)]
    for (int i = 0; i < 16;) {
      const int jb = rb + 4 * i;
      if (jb >= m) break;
      // rows past the pair's first 128 (and below m) need no masks (as in k_hist_pair32)
      auto iteration = [&](auto tag, auto nh, auto nr) {
        constexpr int RR = decltype(nr)::value;   // rows in this iteration
        constexpr int MM = decltype(tag)::value;   // masks: 0 none, 1 the second strip's only, 2 all
        constexpr bool MASKED = MM == 2;
        constexpr int NH = decltype(nh)::value;   // strips of the pair with work in these rows
        cplx G[RR][2][C];
#pragma unroll
        for (int r = 0; r < RR; ++r)
#pragma unroll
          for (int h = 0; h < NH; ++h) {
            int j = jb + 4 * r;
            bool v = (MM == 2 || (MM == 1 && h == 1)) ? (colv[h] && tp[h] <= j && j < m) : true;
            const cplx* row = hk[h] + 64 * (int64_t)C * j;
#pragma unroll
            for (int c = 0; c < C; ++c) G[r][h][c] = v ? load_stream(row + 64 * c) : czero();
          }
        double rt[RR][2 * NBB];
#pragma unroll
        for (int r = 0; r < RR; ++r) {
          int j = jb + 4 * r;
          int jc = MASKED ? (j < m ? j : m - 1) : j;
          cplx SR[NBB];
#pragma unroll
          for (int e = 0; e < NBB; ++e) SR[e] = sk[(2 * NBB + e) * d.Tp + jc];
#pragma unroll
          for (int e = 0; e < 2 * NBB; ++e) rt[r][e] = 0.0;
#pragma unroll
          for (int h = 0; h < NH; ++h) {
            mm_acc<NB>(acc[h], SR, G[r][h]);
            mm_acc<NB>(acc[h] + NBB, SR, G[r][h] + NBB);
            cplx Sl[NBB], Sg[NBB], a[NBB], u[NBB];
#pragma unroll
            for (int e = 0; e < NBB; ++e) {
              Sl[e] = sS[h][0][e][lane];
              Sg[e] = sS[h][1][e][lane];
            }
            mat_zero<NB>(a);
            mat_zero<NB>(u);
            mm_acc_bdag<NB>(a, Sl, G[r][h] + NBB);
            mm_acc_bdag<NB>(u, Sg, G[r][h]);
            bool rv = (MM == 2 || (MM == 1 && h == 1)) ? tp[h] < j : true;
#pragma unroll
            for (int e = 0; e < NBB; ++e) {
              rt[r][2 * e] += rv ? a[e].x - u[e].x : 0.0;
              rt[r][2 * e + 1] += rv ? a[e].y - u[e].y : 0.0;
            }
          }
        }
        if constexpr (RR == 1 && NBB == 4) {
          // one row, four components: each component's (re, im) is one group of a 4-group
          // reduce-scatter (2 lane reductions instead of 8)
          double xg[4][2];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            xg[e][0] = rt[0][2 * e];
            xg[e][1] = rt[0][2 * e + 1];
          }
          reduce_rows<4>(xg);
          int e = reduced_row<4>(lane);
          if (e >= 0) st[e * ROWS_ST + (jb - cb)] = cmk(xg[0][0], xg[0][1]);
        } else {
          reduce_rows<RR>(rt);
          int rr = reduced_row<RR>(lane);
          if (rr >= 0) {
#pragma unroll
            for (int e = 0; e < NBB; ++e) st[e * ROWS_ST + (jb - cb) + 4 * rr] = cmk(rt[0][2 * e], rt[0][2 * e + 1]);
          }
        }
      };
      // rows of the pair's first 64 lie above every column of its second strip: one strip's
      // work; in its next 64 rows every column of the first strip lies below the row: masks for
      // the second strip only
      // (an iteration's rows jb, jb + 4, ..., jb + 4 (RR - 1) lie in one 64-row chunk)
      if (jb >= 128 * sp + 128 && jb + 4 * (R - 1) < m) {
        iteration(IntTag<0>{}, IntTag<2>{}, IntTag<R>{});
        i += R;
      } else if (R == 1 && jb + 4 < 128 * sp + 64 && jb + 4 < m) {
        // two rows at a time where only the first strip has work: its loads of both rows in
        // flight together (one row would keep half the loads of a full iteration in flight)
        iteration(IntTag<2>{}, IntTag<1>{}, IntTag<2>{});
        i += 2;
      } else if (jb + 4 * (R - 1) < 128 * sp + 64) {
        iteration(IntTag<2>{}, IntTag<1>{}, IntTag<R>{});
        i += R;
      } else if (jb >= 128 * sp + 64 && jb + 4 * (R - 1) < m && jb + 4 * (R - 1) < 128 * sp + 128) {
        iteration(IntTag<1>{}, IntTag<2>{}, IntTag<R>{});
        i += R;
      } else {
        iteration(IntTag<2>{}, IntTag<2>{}, IntTag<R>{});
        i += R;
      }
    }
    // every fourth chunk (and the last): the staged rows of all four wavefronts leave as one
    // contiguous run of up to 256 rows per component (4 KB), streaming stores
    if (cslot == ROWS_ST / 64 - 1 || cb + 64 >= m) {
      __syncthreads();
      const int base = cb - 64 * cslot;
      const int nrows = (cb + 64 < m ? cb + 64 : m) - base;
      for (int q = threadIdx.x; q < NBB * nrows; q += 256) {
        const int e = q / nrows, row = q - e * nrows;
        store_stream(rp + (int64_t)e * d.Tp + base + row, stg[e][row]);
      }
      __syncthreads();
    }
  }
  // combine the 4 wavefronts' column sums, strip by strip
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (wv > 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) red[wv - 1][c][lane] = acc[h][c];
    }
    __syncthreads();
    if (wv == 0 && colv[h]) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        cplx a = acc[h][c];
        a = cadd(a, red[0][c][lane]);
        a = cadd(a, red[1][c][lane]);
        a = cadd(a, red[2][c][lane]);
        colsum[rowbuf_idx(d, k, c, tp[h])] = a;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ history sums, FP32 form
// Same structure as k_hist_pair over an FP32-stored history (complex64, half the bytes, a
// column's component pairs in one 16-byte load): R = 2 rows per iteration at nb = 2 (2 rows x
// 2 strips x 4 loads in flight per wavefront), R = 4 at nb = 1. Products and the 64-lane row
// reductions in FP32; the column sums accumulate in FP32 over each wavefront's 16 rows of a
// 64-row chunk and are then added into FP64 registers; row partials and column sums leave the
// kernel in FP64 (the cross-strip reduction, the end points, the update and the density matrix
// stay FP64).
template <int NB>
__global__ __launch_bounds__(256) void k_hist_pair32(Dims d, const cplx32* __restrict__ hist,
                                                     const cplx* __restrict__ sig, cplx* __restrict__ colsum,
                                                     cplx* __restrict__ rowpart, int m) {
  constexpr int NBB = NB * NB, C = 2 * NBB;
  constexpr int R = NB == 1 ? 4 : 2;
  __shared__ cplx red[3][C][64];
  constexpr int ROWS_ST = 256;   // row partials staged over four 64-row chunks, as in k_hist_pair
  __shared__ cplx stg[NBB][ROWS_ST];
  __shared__ cplx32 sS[2][2][NBB][64];
  const int sp = blockIdx.x / d.nk;
  const int k = blockIdx.x - sp * d.nk;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const cplx* sk = sig + (int64_t)k * 3 * NBB * d.Tp;
  for (int q = threadIdx.x; q < 4 * NBB * 64; q += 256) {
    int l = q & 63, e = (q >> 6) % NBB, x = (q >> 6) / NBB;
    int t = 64 * (2 * sp + (x >> 1)) + l;
    sS[x >> 1][x & 1][e][l] = to32(t < m ? sk[((x & 1) * NBB + e) * d.Tp + t] : czero());
  }
  __syncthreads();
  const bool two = 64 * (2 * sp + 1) < m;
  int tp[2];
  bool colv[2];
  const cplx32* hk[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    tp[h] = 64 * (2 * sp + h) + lane;
    colv[h] = tp[h] < m;
    hk[h] = hist + strip_lane_base(d, k, (h && two) ? 2 * sp + 1 : 2 * sp, lane);
  }
  cplx acc[2][C];
  cplx32 acc32[2][C];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int c = 0; c < C; ++c) {
      acc[h][c] = czero();
      acc32[h][c] = make_float2(0.f, 0.f);
    }
  cplx* rp = const_cast<cplx*>(rowpart_slot(d, rowpart, k, sp));
  for (int cb = 128 * sp; cb < m; cb += 64) {
    const int rb = cb + wv;   // the wavefront's rows of the chunk: rb, rb + 4, ..., rb + 60
    const int cslot = ((cb - 128 * sp) >> 6) % (ROWS_ST / 64);
    cplx* st = &stg[0][64 * cslot];   // st[e * ROWS_ST + (row - cb)]
    for (int i = 0; i < 16 / R; ++i) {
      const int jb = rb + 4 * R * i;
      if (jb >= m) break;
      // rows past the pair's first 128 (and below m) need no masks: every lane's columns lie
      // below the row, so that common case runs without the bounds selects
      auto iteration = [&](auto tag, auto nh) {
        constexpr int MM = decltype(tag)::value;   // masks: 0 none, 1 the second strip's only, 2 all
        constexpr bool MASKED = MM == 2;
        constexpr int NH = decltype(nh)::value;   // strips of the pair with work in these rows
        cplx32 G[R][2][C];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int h = 0; h < NH; ++h) {
            int j = jb + 4 * r;
            bool v = (MM == 2 || (MM == 1 && h == 1)) ? (colv[h] && tp[h] <= j && j < m) : true;
            const cplx32* row = hk[h] + 64 * (int64_t)C * j;
#pragma unroll
            for (int c2 = 0; c2 < C / 2; ++c2) {
              if (v) {
                load_stream32x2(row + 128 * c2, G[r][h][2 * c2], G[r][h][2 * c2 + 1]);
              } else {
                G[r][h][2 * c2] = make_float2(0.f, 0.f);
                G[r][h][2 * c2 + 1] = make_float2(0.f, 0.f);
              }
            }
          }
        float rt[R][2 * NBB];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          int j = jb + 4 * r;
          int jc = MASKED ? (j < m ? j : m - 1) : j;
          cplx32 SR[NBB];
#pragma unroll
          for (int e = 0; e < NBB; ++e) SR[e] = to32(sk[(2 * NBB + e) * d.Tp + jc]);
#pragma unroll
          for (int e = 0; e < 2 * NBB; ++e) rt[r][e] = 0.f;
#pragma unroll
          for (int h = 0; h < NH; ++h) {
#pragma unroll
            for (int sc = 0; sc < 2; ++sc)
#pragma unroll
              for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                  for (int l = 0; l < NB; ++l)
                    cmac32(acc32[h][sc * NBB + a * NB + b], SR[a * NB + l], G[r][h][sc * NBB + l * NB + b]);
            bool rv = (MM == 2 || (MM == 1 && h == 1)) ? tp[h] < j : true;
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
              for (int b = 0; b < NB; ++b) {
                cplx32 x = make_float2(0.f, 0.f), u = make_float2(0.f, 0.f);
#pragma unroll
                for (int l = 0; l < NB; ++l) {
                  cmacc32(x, sS[h][0][a * NB + l][lane], G[r][h][NBB + b * NB + l]);
                  cmacc32(u, sS[h][1][a * NB + l][lane], G[r][h][b * NB + l]);
                }
                int e = a * NB + b;
                rt[r][2 * e] += rv ? x.x - u.x : 0.f;
                rt[r][2 * e + 1] += rv ? x.y - u.y : 0.f;
              }
          }
        }
        if constexpr (R == 2 && NBB == 4) {
          // two rows, four components: groups (row, component pair) of a 4-group reduce-scatter
          // (4 lane reductions instead of 8); group g = 2 r + p holds components 2 p, 2 p + 1
          float xg[4][4];
#pragma unroll
          for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int p2 = 0; p2 < 2; ++p2)
#pragma unroll
              for (int q = 0; q < 4; ++q) xg[2 * r + p2][q] = rt[r][4 * p2 + q];
          reduce_rows32<4>(xg);
          int g = reduced_row<4>(lane);
          if (g >= 0) {
            int r = g >> 1, p2 = g & 1;
#pragma unroll
            for (int c = 0; c < 2; ++c)
              st[(2 * p2 + c) * ROWS_ST + (jb - cb) + 4 * r] = cmk((double)xg[0][2 * c], (double)xg[0][2 * c + 1]);
          }
        } else {
          reduce_rows32<R>(rt);
          int rr = reduced_row<R>(lane);
          if (rr >= 0) {
#pragma unroll
            for (int e = 0; e < NBB; ++e)
              st[e * ROWS_ST + (jb - cb) + 4 * rr] = cmk((double)rt[0][2 * e], (double)rt[0][2 * e + 1]);
          }
        }
      };
      // rows of the pair's first 64 lie above every column of its second strip: one strip's
      // work; in its next 64 rows every column of the first strip lies below the row: masks for
      // the second strip only
      // (an iteration's rows jb, jb + 4, ..., jb + 4 (R - 1) lie in one 64-row chunk)
      if (jb >= 128 * sp + 128 && jb + 4 * (R - 1) < m)
        iteration(IntTag<0>{}, IntTag<2>{});
      else if (jb + 4 * (R - 1) < 128 * sp + 64)
        iteration(IntTag<2>{}, IntTag<1>{});
      else if (jb >= 128 * sp + 64 && jb + 4 * (R - 1) < m && jb + 4 * (R - 1) < 128 * sp + 128)
        iteration(IntTag<1>{}, IntTag<2>{});
      else
        iteration(IntTag<2>{}, IntTag<2>{});
    }
    // the group's FP32 column sums into the FP64 accumulators
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        acc[h][c].x += (double)acc32[h][c].x;
        acc[h][c].y += (double)acc32[h][c].y;
        acc32[h][c] = make_float2(0.f, 0.f);
      }
    if (cslot == ROWS_ST / 64 - 1 || cb + 64 >= m) {
      __syncthreads();
      const int base = cb - 64 * cslot;
      const int nrows = (cb + 64 < m ? cb + 64 : m) - base;
      for (int q = threadIdx.x; q < NBB * nrows; q += 256) {
        const int e = q / nrows, row = q - e * nrows;
        store_stream(rp + (int64_t)e * d.Tp + base + row, stg[e][row]);
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (wv > 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) red[wv - 1][c][lane] = acc[h][c];
    }
    __syncthreads();
    if (wv == 0 && colv[h]) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        cplx a = acc[h][c];
        a = cadd(a, red[0][c][lane]);
        a = cadd(a, red[1][c][lane]);
        a = cadd(a, red[2][c][lane]);
        colsum[rowbuf_idx(d, k, c, tp[h])] = a;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ history sums, nb = 3
// One 64-column strip per block (row partials in slot s), every wavefront over every fourth
// row; the 18 components of a block leave no registers for a second strip. FP64: one row per
// iteration, the per-column Sigma of the row term in LDS. Row partials stored by lane 0.
template <int NB>
__global__ __launch_bounds__(256) void k_hist_bulk(Dims d, const cplx* __restrict__ hist,
                                                   const cplx* __restrict__ sig, cplx* __restrict__ colsum,
                                                   cplx* __restrict__ rowpart, int m) {
  constexpr int NBB = NB * NB, C = 2 * NBB;
  constexpr int CH = (C < 8) ? C : 8;  // components per LDS combine round
  __shared__ cplx red[3][CH][64];
  __shared__ cplx sS[2][NBB][64];
  int s = blockIdx.x / d.nk;  // strips with the most rows first
  int k = blockIdx.x - s * d.nk;
  int lane = threadIdx.x & 63;
  int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int tp = 64 * s + lane;
  bool colv = tp < m;
  const cplx* sk = sig + (int64_t)k * 3 * NBB * d.Tp;
  for (int i = threadIdx.x; i < 2 * NBB * 64; i += 256) {
    int x = i / (NBB * 64), e = (i / 64) % NBB, l = i % 64;
    int t = 64 * s + l;
    sS[x][e][l] = t < m ? sk[(x * NBB + e) * d.Tp + t] : czero();
  }
  __syncthreads();
  cplx acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = czero();
  const cplx* hk = hist + strip_lane_base(d, k, s, lane);
  cplx* rp = const_cast<cplx*>(rowpart_slot(d, rowpart, k, s));
  for (int j = 64 * s + wv; j < m; j += 4) {
    bool v = colv && tp <= j;
    const cplx* row = hk + 64 * (int64_t)C * j;
    cplx G[C];
#pragma unroll
    for (int c = 0; c < C; ++c) G[c] = v ? load_stream(row + 64 * c) : czero();
    cplx SR[NBB];
#pragma unroll
    for (int e = 0; e < NBB; ++e) SR[e] = sk[(2 * NBB + e) * d.Tp + j];
    mm_acc<NB>(acc, SR, G);
    mm_acc<NB>(acc + NBB, SR, G + NBB);
    bool rv = tp < j;
    double rt[1][2 * NBB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        cplx x = czero(), u = czero();
#pragma unroll
        for (int l = 0; l < NB; ++l) {
          cmacc(x, sS[0][a * NB + l][lane], G[NBB + b * NB + l]);
          cmacc(u, sS[1][a * NB + l][lane], G[b * NB + l]);
        }
        int e = a * NB + b;
        rt[0][2 * e] = rv ? x.x - u.x : 0.0;
        rt[0][2 * e + 1] = rv ? x.y - u.y : 0.0;
      }
    reduce_rows<1>(rt);
    if (lane == 0) {
#pragma unroll
      for (int e = 0; e < NBB; ++e) rp[(int64_t)e * d.Tp + j] = cmk(rt[0][2 * e], rt[0][2 * e + 1]);
    }
  }
  // combine the 4 wavefronts' column sums
#pragma unroll
  for (int c0 = 0; c0 < C; c0 += CH) {
    if (wv > 0) {
#pragma unroll
      for (int c = 0; c < CH; ++c) red[wv - 1][c][lane] = acc[c0 + c];
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        cplx a = acc[c0 + c];
        a = cadd(a, red[0][c][lane]);
        a = cadd(a, red[1][c][lane]);
        a = cadd(a, red[2][c][lane]);
        if (colv) colsum[rowbuf_idx(d, k, c0 + c, tp)] = a;
      }
    }
    __syncthreads();
  }
}

// FP32 form at nb = 3: two rows per iteration, Sigma of the row term in registers; FP32 tiles
// of 16 rows per wavefront added into FP64 accumulators.
template <int NB>
__global__ __launch_bounds__(256) void k_hist_bulk32(Dims d, const cplx32* __restrict__ hist,
                                                     const cplx* __restrict__ sig, cplx* __restrict__ colsum,
                                                     cplx* __restrict__ rowpart, int m) {
  constexpr int NBB = NB * NB, C = 2 * NBB;
  constexpr int CH = (C < 8) ? C : 8;
  constexpr int R = 2;
  constexpr int FLUSH = 16 / R;  // iterations per FP32 accumulation tile (16 rows)
  __shared__ cplx red[3][CH][64];
  int s = blockIdx.x / d.nk;
  int k = blockIdx.x - s * d.nk;
  int lane = threadIdx.x & 63;
  int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int tp = 64 * s + lane;
  bool colv = tp < m;
  const cplx* sk = sig + (int64_t)k * 3 * NBB * d.Tp;
  cplx32 Sl[NBB], Sg[NBB];
#pragma unroll
  for (int e = 0; e < NBB; ++e) {
    Sl[e] = to32(colv ? sk[(0 * NBB + e) * d.Tp + tp] : czero());
    Sg[e] = to32(colv ? sk[(1 * NBB + e) * d.Tp + tp] : czero());
  }
  cplx acc[C];
  cplx32 acc32[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    acc[c] = czero();
    acc32[c] = make_float2(0.f, 0.f);
  }
  const cplx32* hk = hist + strip_lane_base(d, k, s, lane);
  cplx* rp = const_cast<cplx*>(rowpart_slot(d, rowpart, k, s));
  int it = 0;
  for (int jb = 64 * s + R * wv; jb < m; jb += 4 * R) {
    cplx32 G[R][C];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int j = jb + r;
      bool v = colv && tp <= j && j < m;
      const cplx32* row = hk + 64 * (int64_t)C * j;
#pragma unroll
      for (int c2 = 0; c2 < C / 2; ++c2) {
        if (v) {
          load_stream32x2(row + 128 * c2, G[r][2 * c2], G[r][2 * c2 + 1]);
        } else {
          G[r][2 * c2] = make_float2(0.f, 0.f);
          G[r][2 * c2 + 1] = make_float2(0.f, 0.f);
        }
      }
    }
    float rt[R][2 * NBB];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int j = jb + r;
      int jc = j < m ? j : m - 1;
      cplx32 SR[NBB];
#pragma unroll
      for (int e = 0; e < NBB; ++e) SR[e] = to32(sk[(2 * NBB + e) * d.Tp + jc]);
#pragma unroll
      for (int sc = 0; sc < 2; ++sc)
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
          for (int jj = 0; jj < NB; ++jj)
#pragma unroll
            for (int l = 0; l < NB; ++l) cmac32(acc32[sc * NBB + i * NB + jj], SR[i * NB + l], G[r][sc * NBB + l * NB + jj]);
      bool rv = tp < j;
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int jj = 0; jj < NB; ++jj) {
          cplx32 a = make_float2(0.f, 0.f), u = make_float2(0.f, 0.f);
#pragma unroll
          for (int l = 0; l < NB; ++l) {
            cmacc32(a, Sl[i * NB + l], G[r][NBB + jj * NB + l]);
            cmacc32(u, Sg[i * NB + l], G[r][jj * NB + l]);
          }
          int e = i * NB + jj;
          rt[r][2 * e] = rv ? a.x - u.x : 0.f;
          rt[r][2 * e + 1] = rv ? a.y - u.y : 0.f;
        }
    }
    if (++it == FLUSH) {
      it = 0;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        acc[c].x += (double)acc32[c].x;
        acc[c].y += (double)acc32[c].y;
        acc32[c] = make_float2(0.f, 0.f);
      }
    }
    reduce_rows32<R>(rt);
    int rsel = reduced_row<R>(lane);
    if (rsel >= 0 && jb + rsel < m) {
#pragma unroll
      for (int e = 0; e < NBB; ++e)
        rp[(int64_t)e * d.Tp + jb + rsel] = cmk((double)rt[0][2 * e], (double)rt[0][2 * e + 1]);
    }
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    acc[c].x += (double)acc32[c].x;
    acc[c].y += (double)acc32[c].y;
  }
#pragma unroll
  for (int c0 = 0; c0 < C; c0 += CH) {
    if (wv > 0) {
#pragma unroll
      for (int c = 0; c < CH; ++c) red[wv - 1][c][lane] = acc[c0 + c];
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        cplx a = acc[c0 + c];
        a = cadd(a, red[0][c][lane]);
        a = cadd(a, red[1][c][lane]);
        a = cadd(a, red[2][c][lane]);
        if (colv) colsum[rowbuf_idx(d, k, c0 + c, tp)] = a;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ history sums, nb = 4
// With nb = 4 a stored block has 2 nb^2 = 32 components, too many for one wavefront's
// registers next to its column sums. The block's components are split by half: waves 0 and 2
// stream G^< (components 0..15), waves 1 and 3 stream G^> (16..31); the row pair (0, 1) takes
// rows 0-15 of every 32-row chunk of the strip, the pair (2, 3) rows 16-31 (16 contiguous 1 KB
// segments in flight per wavefront). Half 0 contributes -Sigma^>_{t'} (G^<_{j t'})^dag to the
// row term, half 1 +Sigma^<_{t'} (G^>_{j t'})^dag. The four block rows of a row term go through
// one 64-lane reduce-scatter together (4 quantities for the instructions of one); a
// wavefront's 16 row partials are staged in LDS (two buffers, alternating by chunk), and after
// one block barrier per 32-row chunk the two halves' partials are added and stored as 256-byte
// runs with streaming stores, one row-partial slot per strip. The per-column Sigma of the row
// term is read from LDS. FP64 storage; 2 waves per SIMD.
template <int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_hist_bulk_split(
    Dims d, const cplx* __restrict__ hist, const cplx* __restrict__ sig, cplx* __restrict__ colsum,
    cplx* __restrict__ rowpart, int m) {
  constexpr int NBB = NB * NB, C = 2 * NBB;
  static_assert(NB == 4, "the four block rows share one reduce-scatter");
  __shared__ cplx sS[2][NBB][64];  // [half][e][lane]: half 0 needs Sigma^>, half 1 Sigma^<;
                                   // reused for the column-sum combine after the row loop
  __shared__ cplx stg[2][2][2][NBB * 16];  // [buffer][row pair][half][e * 16 + row]
  int s = blockIdx.x / d.nk;
  int k = blockIdx.x - s * d.nk;
  int lane = threadIdx.x & 63;
  int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform: rows and Sigma^R in SGPRs
  int h = wv & 1, rg = wv >> 1;
  int tp = 64 * s + lane;
  bool colv = tp < m;
  const cplx* sk = sig + (int64_t)k * 3 * NBB * d.Tp;
  for (int i = threadIdx.x; i < 2 * NBB * 64; i += 256) {
    int x = i / (NBB * 64), e = (i / 64) % NBB, l = i % 64;
    int t = 64 * s + l;
    sS[x][e][l] = t < m ? sk[((1 - x) * NBB + e) * d.Tp + t] : czero();
  }
  __syncthreads();
  cplx acc[NBB];
#pragma unroll
  for (int e = 0; e < NBB; ++e) acc[e] = czero();
  const cplx* hk = hist + strip_lane_base(d, k, s, lane) + 64 * NBB * h;
  cplx* rp = const_cast<cplx*>(rowpart_slot(d, rowpart, k, s));
  const double sgn = h ? 1.0 : -1.0;
  int buf = 0;
  for (int cb = 64 * s; cb < m; cb += 32) {  // the same chunks in every wavefront
    const int rb = cb + 16 * rg;
    cplx* st = stg[buf][rg][h];
    for (int i = 0; i < 16; ++i) {
      const int j = rb + i;
      if (j >= m) break;
      bool v = colv && tp <= j;
      const cplx* row = hk + 64 * (int64_t)C * j;
      cplx G[NBB];
#pragma unroll
      for (int e = 0; e < NBB; ++e) G[e] = v ? load_stream(row + 64 * e) : czero();
      bool rv = tp < j;
      double x[NB][2 * NB];  // row term of block row a, column b: x[a][2 b], x[a][2 b + 1]
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        cplx SRa[NB];
#pragma unroll
        for (int l = 0; l < NB; ++l) SRa[l] = sk[(2 * NBB + a * NB + l) * d.Tp + j];
        // column term, block row a:  acc[a][b] += sum_l SR[a][l] G[l][b]
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int l = 0; l < NB; ++l) cmac(acc[a * NB + b], SRa[l], G[l * NB + b]);
        // row term, block row a:  sgn * sum_l S[a][l] conj(G[b][l])
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          cplx t = czero();
#pragma unroll
          for (int l = 0; l < NB; ++l) cmacc(t, sS[h][a * NB + l][lane], G[b * NB + l]);
          x[a][2 * b] = rv ? sgn * t.x : 0.0;
          x[a][2 * b + 1] = rv ? sgn * t.y : 0.0;
        }
      }
      reduce_rows<NB>(x);
      int ra = reduced_row<NB>(lane);
      if (ra >= 0) {
#pragma unroll
        for (int b = 0; b < NB; ++b) st[(ra * NB + b) * 16 + i] = cmk(x[0][2 * b], x[0][2 * b + 1]);
      }
    }
    __syncthreads();  // both halves of the chunk staged; the other buffer is free again
    flush_rows_fold<NBB>(stg[buf][rg][0], stg[buf][rg][1], rp, d.Tp, rb, m, lane, h);
    buf ^= 1;
  }
  __syncthreads();  // every wavefront is done with sS
  cplx (*red)[NBB][64] = sS;
  if (rg == 1) {
#pragma unroll
    for (int e = 0; e < NBB; ++e) red[h][e][lane] = acc[e];
  }
  __syncthreads();
  if (rg == 0 && colv) {
#pragma unroll
    for (int e = 0; e < NBB; ++e) colsum[rowbuf_idx(d, k, h * NBB + e, tp)] = cadd(acc[e], red[h][e][lane]);
  }
}

// FP32 form of k_hist_bulk_split: each half's 16 components are 8 column-interleaved pairs,
// one 16-byte load each; FP32 products and row reductions, column sums in FP32 over each
// wavefront's 16 rows of a 32-row chunk, then FP64. The row pair (0, 1) takes the even rows of
// every 32-row chunk and (2, 3) the odd ones, so a chunk cut short by m keeps both pairs busy, and
// the whole block stores a chunk's row partials as 512-byte runs (this kernel is bound by the
// vector ALU; the FP64 kernel's stream ran 1.7 % slower with interleaved rows and keeps 16
// consecutive rows per pair).
template <int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_hist_bulk32_split(
    Dims d, const cplx32* __restrict__ hist, const cplx* __restrict__ sig, cplx* __restrict__ colsum,
    cplx* __restrict__ rowpart, int m) {
  constexpr int NBB = NB * NB, C = 2 * NBB;
  static_assert(NB == 4, "the four block rows share one reduce-scatter");
  static_assert(NBB % 2 == 0, "component pairs must not straddle the halves");
  __shared__ cplx32 sS[2][NBB][64];
  __shared__ cplx stg[2][2][NBB * 32];  // [buffer][half][e * 32 + row - cb]; column-sum combine
                                        // after the row loop
  int s = blockIdx.x / d.nk;
  int k = blockIdx.x - s * d.nk;
  int lane = threadIdx.x & 63;
  int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int h = wv & 1, rg = wv >> 1;
  int tp = 64 * s + lane;
  bool colv = tp < m;
  const cplx* sk = sig + (int64_t)k * 3 * NBB * d.Tp;
  for (int i = threadIdx.x; i < 2 * NBB * 64; i += 256) {
    int x = i / (NBB * 64), e = (i / 64) % NBB, l = i % 64;
    int t = 64 * s + l;
    sS[x][e][l] = to32(t < m ? sk[((1 - x) * NBB + e) * d.Tp + t] : czero());
  }
  __syncthreads();
  cplx acc[NBB];
  cplx32 acc32[NBB];
#pragma unroll
  for (int e = 0; e < NBB; ++e) {
    acc[e] = czero();
    acc32[e] = make_float2(0.f, 0.f);
  }
  const cplx32* hk = hist + strip_lane_base(d, k, s, lane) + 64 * NBB * h;
  cplx* rp = const_cast<cplx*>(rowpart_slot(d, rowpart, k, s));
  const float sgn = h ? 1.f : -1.f;
  int buf = 0;
  for (int cb = 64 * s; cb < m; cb += 32) {  // the same chunks in every wavefront
    const int rb = cb + rg;   // the wave pair's rows of the chunk: rb, rb + 2, ..., rb + 30
    cplx* st = stg[buf][h];
    // groups of 16 rows past the strip's first 64 rows and below m need no masks (this
    // kernel is bound by the vector ALU; the FP64 kernel keeps one path, a second one would
    // not fit its registers)
    auto rows16 = [&](auto tag) {
      constexpr bool MASKED = decltype(tag)::value;
      for (int i = 0; i < 16; ++i) {
        const int j = rb + 2 * i;
        if (MASKED && j >= m) break;
        bool v = MASKED ? (colv && tp <= j) : true;
        const cplx32* row = hk + 64 * (int64_t)C * j;
        cplx32 G[NBB];
#pragma unroll
        for (int p = 0; p < NBB / 2; ++p) {
          if (v) {
            load_stream32x2(row + 128 * p, G[2 * p], G[2 * p + 1]);
          } else {
            G[2 * p] = make_float2(0.f, 0.f);
            G[2 * p + 1] = make_float2(0.f, 0.f);
          }
        }
        bool rv = MASKED ? tp < j : true;
        float x[NB][2 * NB];
#pragma unroll
        for (int a = 0; a < NB; ++a) {
          cplx32 SRa[NB];
#pragma unroll
          for (int l = 0; l < NB; ++l) SRa[l] = to32(sk[(2 * NBB + a * NB + l) * d.Tp + j]);
#pragma unroll
          for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int l = 0; l < NB; ++l) cmac32(acc32[a * NB + b], SRa[l], G[l * NB + b]);
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            cplx32 t = make_float2(0.f, 0.f);
#pragma unroll
            for (int l = 0; l < NB; ++l) cmacc32(t, sS[h][a * NB + l][lane], G[b * NB + l]);
            x[a][2 * b] = rv ? sgn * t.x : 0.f;
            x[a][2 * b + 1] = rv ? sgn * t.y : 0.f;
          }
        }
        reduce_rows32<NB>(x);
        int ra = reduced_row<NB>(lane);
        if (ra >= 0) {
#pragma unroll
          for (int b = 0; b < NB; ++b) st[(ra * NB + b) * 32 + (j - cb)] = cmk((double)x[0][2 * b], (double)x[0][2 * b + 1]);
        }
      }
    };
    if (rb >= 64 * s + 64 && rb + 30 < m)
      rows16(BoolTag<false>{});
    else
      rows16(BoolTag<true>{});
#pragma unroll
    for (int e = 0; e < NBB; ++e) {
      acc[e].x += (double)acc32[e].x;
      acc[e].y += (double)acc32[e].y;
      acc32[e] = make_float2(0.f, 0.f);
    }
    __syncthreads();  // both halves of the chunk staged; the other buffer is free again
    flush_chunk_fold<NBB>(stg[buf][0], stg[buf][1], rp, d.Tp, cb, m);
    buf ^= 1;
  }
  __syncthreads();  // every wavefront is done with stg
  cplx (*red)[NBB][64] = reinterpret_cast<cplx (*)[NBB][64]>(&stg[0][0][0]);
  if (rg == 1) {
#pragma unroll
    for (int e = 0; e < NBB; ++e) red[h][e][lane] = acc[e];
  }
  __syncthreads();
  if (rg == 0 && colv) {
#pragma unroll
    for (int e = 0; e < NBB; ++e) colsum[rowbuf_idx(d, k, h * NBB + e, tp)] = cadd(acc[e], red[h][e][lane]);
  }
}

// ------------------------------------------------------------------ history sums, FP32-MFMA form
// The same sums as above on the quad layout of the FP32-MFMA form. A block takes strip s of one
// k; its wavefronts split the 64 columns into 4 groups g of 16 (and, at nb = 4, the components
// into their G^< and G^> halves: 8 wavefronts; at nb <= 3 each wavefront takes both halves: 4).
// Per quad of 4 rows a lane L holds the pair (j = j0 + L / 16, t' = 16 g + L % 16):
// * column term, on the matrix cores: for component (half, b) the 16 x 16 tile
//     D[m][t'] += sum_{r < 4} A_l^ri[m][r] G_{l b}^ri(j0 + r, t'),   m = (hi/lo, a, re/im),
//   one v_mfma_f32_16x16x4f32 per (l, re/im) with K = the quad's 4 rows: A holds the real
//   embedding of Sigma^R(t_j)_{a l} (re rows: [Re, -Im]; im rows: [Im, Re]) split into its FP32
//   high part and the FP32 rounding of the remainder (rows m < 2 nb: high, 2 nb <= m < 4 nb: low),
//   so the two compensated products fill the 16-row tile at nb = 4 and are added in FP64 at the
//   end. The tiles accumulate in FP32 over one chunk of quads (8 quads = 32 rows at nb = 4, 16
//   quads = 64 rows otherwise), then into FP64 registers. The A operands of a chunk are split and
//   staged in LDS once per block, one chunk ahead, by all its threads (every wavefront of the block
//   needs the same rows).
// * row term, on the vector ALU in FP32: each lane forms sgn Sigma^{>,<}_{t'} (G_{j t'})^dag of its
//   pair; a DPP reduce-scatter over the 16 lanes of each row (four rows at once) leaves one
//   component per lane; the wavefronts' partials of a chunk are staged in LDS (two buffers) and,
//   after one block barrier per chunk, added in a fixed order in FP64 and stored to the strip's
//   row-partial slot with streaming stores (at nb <= 2 staged over four chunks and stored as
//   4 KB runs).
// Quads past the strip's triangle (its first 16) and below m run without bounds selects. The
// next quad's loads are issued before the current quad is processed, and no load sits behind a
// branch, so the waits for one quad's data are exact.
__device__ __forceinline__ float split_part(double x, bool low) {
  float hi = (float)x;
  return low ? (float)(x - (double)hi) : hi;
}
template <int CTRL, int CNT>
__device__ __forceinline__ void rs16_step(float* x, bool upper) {
  if constexpr (CNT >= 2) {
    constexpr int H = CNT / 2;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      float keep = upper ? x[i + H] : x[i];
      float send = upper ? x[i] : x[i + H];
      x[i] = keep + dpp_f<CTRL>(send);
    }
  } else {
    x[0] += dpp_f<CTRL>(x[0]);
  }
}
// Reduce-scatter of VP values (a power of two) over the 16 lanes of each row: partners differ in
// bit 3 (row mirror), bit 2 (half-row mirror), bit 1 and bit 0 (quad permutations) of the lane.
// Afterwards lane l of a row holds the row sums of values (VP / 16) l .. (VP / 16) l + VP / 16 - 1
// in x[0 ..] if VP >= 16, else of value l / (16 / VP) in x[0].
template <int VP>
__device__ __forceinline__ void reduce_scatter16(float (&x)[VP], int lane) {
  rs16_step<0x140, VP>(x, lane & 8);
  rs16_step<0x141, (VP / 2 > 1 ? VP / 2 : 1)>(x, lane & 4);
  rs16_step<0x4E, (VP / 4 > 1 ? VP / 4 : 1)>(x, lane & 2);
  rs16_step<0xB1, (VP / 8 > 1 ? VP / 8 : 1)>(x, lane & 1);
}

template <int NB>
struct MfmaShape {
  static constexpr int NBB = NB * NB, C = 2 * NBB;
  static constexpr int HS = NB == 4 ? 1 : 2;          // component halves per wavefront
  static constexpr int WAVES = 4 * (2 / HS);
  static constexpr int NCH = HS == 2 ? NBB : NBB / 2;  // 16-byte loads per lane and quad
  static constexpr int VP = 2 * NBB <= 2 ? 2 : (2 * NBB <= 8 ? 8 : 32);           // row-term values, padded
  static constexpr int CQ = NB == 4 ? 8 : 16;         // quads per staged chunk (32 or 64 rows)
  static constexpr int PF = 1;                        // quads whose loads are in flight ahead
  static constexpr int STAGE = 2 * WAVES * CQ * 4 * VP * 4;  // bytes
  static constexpr int AFR = 2 * CQ * 64 * 2 * NB * 4;       // bytes: A operands of two chunks
  static constexpr int FIN = WAVES * HS * NB * 256 * 8;     // bytes
  // row partials leave in runs of ROWS rows per component: at nb <= 2 the FP64 sums of four
  // 64-row chunks are staged (runs of 4 KB; fewer, longer write bursts in the read stream), at
  // nb >= 3 each chunk's rows are stored directly (a 64-row staging costs more than it saves there)
  static constexpr int ROWS = NB <= 2 ? 256 : 4 * CQ;
  static constexpr int RSTG = NB <= 2 ? NBB * ROWS * 16 : 0;   // bytes
  static constexpr int LDS = (STAGE + AFR) > FIN ? (STAGE + AFR) : FIN;
};

// A operands of the quads of one chunk, [quad][lane][l][re/im] (2 nb floats per lane): lane
// L = 16 r + n of quad q gives row n = (hi/lo, a, re/im) of the real embedding of
// Sigma^R(t_j)_{a l}, j = 64 s + 4 q + r, split into the FP32 high part and the FP32 rounding of
// the remainder; zero outside the 4 nb rows of the tile and for j >= m. Each thread takes
// entries e = tid, tid + block, ...: load() issues the FP64 reads, store() splits and writes.
template <int NB, int NE>
struct AfrFill {
  static_assert(NE * MfmaShape<NB>::WAVES * 64 == MfmaShape<NB>::CQ * 64, "every thread fills NE whole entries");
  cplx x[NE][NB];
  double z[NE];
  // every lane loads a valid entry (row clamped below m); entries outside the tile or past m are
  // zeroed only in store(), so no branch or early use sits behind the loads and the waits for
  // the quads' history loads stay exact
  __device__ __forceinline__ void load(const Dims& d, const cplx* sk, int s, int qfirst, int m, int tid, int nthr) {
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = tid + i * nthr;
      const int L = e & 63, n = L & 15;
      const int j = 64 * s + 4 * (qfirst + (e >> 6)) + (L >> 4);
      z[i] = (n < 4 * NB && j < m) ? 1.0 : 0.0;
      const int aa = (n % (2 * NB)) >> 1;
      const int jl = j < m ? j : m - 1;
#pragma unroll
      for (int l = 0; l < NB; ++l) x[i][l] = sk[(2 * NB * NB + aa * NB + l) * d.Tp + jl];
    }
  }
  __device__ __forceinline__ void store(float* afr, int tid, int nthr) const {
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = tid + i * nthr;
      const int n = e & 15;
      const bool low = n >= 2 * NB, im_row = n & 1;
      float* dst = afr + e * 2 * NB;
#pragma unroll
      for (int l = 0; l < NB; ++l) {
        const float pr = split_part(x[i][l].x * z[i], low), pi = split_part(x[i][l].y * z[i], low);
        dst[2 * l] = im_row ? pi : pr;
        dst[2 * l + 1] = im_row ? pr : -pi;
      }
    }
  }
};

template <int NB>
__global__ __launch_bounds__(MfmaShape<NB>::WAVES * 64) __attribute__((amdgpu_waves_per_eu(2))) void k_hist_mfma(
    Dims d, const float2* __restrict__ hist, const cplx* __restrict__ sig, cplx* __restrict__ colsum,
    cplx* __restrict__ rowpart, int m) {
  using Sh = MfmaShape<NB>;
  constexpr int NBB = Sh::NBB, C = Sh::C, HS = Sh::HS, NCH = Sh::NCH, VP = Sh::VP, CQ = Sh::CQ, WAVES = Sh::WAVES;
  static_assert(HS == 2 || NBB % 2 == 0, "halves must not share a 16-byte load");
  __shared__ __align__(16) unsigned char smem[Sh::LDS];
  constexpr int CPF = Sh::ROWS / (4 * CQ);   // chunks per row-partial store
  __shared__ cplx rstg[Sh::RSTG > 0 ? Sh::RSTG / 16 : 1];
  float* stg = reinterpret_cast<float*>(smem);  // [2][WAVES][CQ][4][VP]
  float* afr = reinterpret_cast<float*>(smem + Sh::STAGE);  // [2][CQ][64][2 nb]
  constexpr int NTHR = WAVES * 64, NE = (CQ * 64 + NTHR - 1) / NTHR;
  const int s = blockIdx.x / d.nk;
  const int k = blockIdx.x - s * d.nk;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = HS == 1 ? (wv >> 1) : wv;
  const int h0 = HS == 1 ? (wv & 1) : 0;   // first component half of this wavefront
  const int r = lane >> 4, n = lane & 15;
  const int tp = 64 * s + 16 * g + n;
  const bool colv = tp < m;
  const cplx* sk = sig + (int64_t)k * 3 * NBB * d.Tp;
  // row-term Sigma of this lane's column: half 0 (G^<) takes -Sigma^>, half 1 (G^>) +Sigma^<
  cplx32 Srow[HS * NBB];
#pragma unroll
  for (int hh = 0; hh < HS; ++hh) {
    const int H = h0 + hh;
    const float sg = H ? 1.f : -1.f;
#pragma unroll
    for (int e = 0; e < NBB; ++e) {
      cplx v = colv ? sk[((1 - H) * NBB + e) * d.Tp + tp] : czero();
      Srow[hh * NBB + e] = make_float2(sg * (float)v.x, sg * (float)v.y);
    }
  }
  typedef float f4 __attribute__((ext_vector_type(4)));
  f4 D[HS][NB];
  double col[HS][NB][4];
#pragma unroll
  for (int hh = 0; hh < HS; ++hh)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      D[hh][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) col[hh][b][v] = 0.0;
    }
  // lane's 16-byte loads of quad q: float4 index (q C 128) + (g C/2 + ci) 64 + lane
  const kbe_f4v* hq = reinterpret_cast<const kbe_f4v*>(hist) +
                      ((int64_t)k * C * d.P + 256 * (int64_t)C * quad_base(s, d.N)) / 2 +
                      (int64_t)(g * (C / 2) + h0 * (NBB / 2)) * 64 + lane;
  const int nq = (m - 64 * s + 3) >> 2;   // quads holding rows below m
  constexpr int PF = Sh::PF, RING = PF + 1;
  static_assert(CQ % RING == 0, "a chunk holds whole turns of the load ring");
  // quad x lives in ring[x % RING]; its loads are issued while quad x - PF is processed
  kbe_f4v ring[RING][NCH];
  // loads are never behind a branch (a quad index past the last is clamped to it), so the
  // waits for one quad's data leave the later quads' loads in flight. Quads q < 4 g lie wholly
  // above the diagonal for this wavefront's columns (16 g .. 16 g + 15 of the strip): their loads
  // are pointed at quad 4 g, which the wavefront reads anyway (cache hits instead of HBM traffic
  // for the unused part of the strip's triangle); the masks zero them.
  const int qlo = 4 * g < nq - 1 ? 4 * g : nq - 1;
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    const int qu = u < qlo ? qlo : (u < nq ? u : nq - 1);
#pragma unroll
    for (int i = 0; i < NCH; ++i) ring[u][i] = __builtin_nontemporal_load(hq + (int64_t)qu * 128 * C + i * 64);
  }
  cplx* rp = const_cast<cplx*>(rowpart_slot(d, rowpart, k, s));
  AfrFill<NB, NE> fill;
  fill.load(d, sk, s, 0, m, threadIdx.x, NTHR);
  fill.store(afr, threadIdx.x, NTHR);
  __syncthreads();
  int buf = 0;
  for (int q0 = 0, ci = 0; q0 < nq; q0 += CQ, ++ci) {
    float* sb = stg + buf * (WAVES * CQ * 4 * VP);
    const float* ab = afr + buf * (CQ * 64 * 2 * NB);
    const bool more = q0 + CQ < nq;
    if (more) fill.load(d, sk, s, q0 + CQ, m, threadIdx.x, NTHR);  // the next chunk's A operands
    for (int qt = 0; qt < CQ; qt += RING) {
#pragma unroll
    for (int u = 0; u < RING; ++u) {
      const int qc = qt + u;
      const int q = q0 + qc;   // quads past the last run masked (all zero), so that every chunk
                               // issues the same loads and the waits at its end stay exact
      {
        const int qn = q + PF < qlo ? qlo : (q + PF < nq ? q + PF : nq - 1);
        const kbe_f4v* nx = hq + (int64_t)qn * 128 * C;
#pragma unroll
        for (int i = 0; i < NCH; ++i) ring[(u + PF) % RING][i] = __builtin_nontemporal_load(nx + i * 64);
      }
      const kbe_f4v* cur = ring[u];
      const int j0 = 64 * s + 4 * q;
      const int j = j0 + r;
      auto quad = [&](auto tag) {
        constexpr bool MASKED = decltype(tag)::value;
        cplx32 G[HS * NBB];
        const bool valid = MASKED ? (colv && tp <= j && j < m) : true;
#pragma unroll
        for (int i = 0; i < NCH; ++i) {
          G[2 * i] = valid ? make_float2(cur[i].x, cur[i].y) : make_float2(0.f, 0.f);
          if (2 * i + 1 < HS * NBB) G[2 * i + 1] = valid ? make_float2(cur[i].z, cur[i].w) : make_float2(0.f, 0.f);
        }
        // A operand of this lane: Sigma^R(t_j)_{a l}, real-embedded and split (staged)
        float Af[NB][2];
        const float* af = ab + (qc * 64 + lane) * 2 * NB;
#pragma unroll
        for (int l = 0; l < NB; ++l) {
          Af[l][0] = af[2 * l];
          Af[l][1] = af[2 * l + 1];
        }
#pragma unroll
        for (int l = 0; l < NB; ++l)
#pragma unroll
          for (int ri = 0; ri < 2; ++ri)
#pragma unroll
            for (int hh = 0; hh < HS; ++hh)
#pragma unroll
              for (int b = 0; b < NB; ++b) {
                const cplx32 gv = G[hh * NBB + l * NB + b];
                D[hh][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(Af[l][ri], ri ? gv.y : gv.x, D[hh][b], 0, 0, 0);
              }
        // row term of this lane's pair
        float x[VP];
#pragma unroll
        for (int i = 0; i < VP; ++i) x[i] = 0.f;
#pragma unroll
        for (int hh = 0; hh < HS; ++hh)
#pragma unroll
          for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              cplx32 t = make_float2(0.f, 0.f);
#pragma unroll
              for (int l = 0; l < NB; ++l) cmacc32(t, Srow[hh * NBB + a * NB + l], G[hh * NBB + b * NB + l]);
              x[2 * (a * NB + b)] += t.x;
              x[2 * (a * NB + b) + 1] += t.y;
            }
        if constexpr (MASKED) {
          const bool rv = tp < j;   // the diagonal belongs to the end-point terms
#pragma unroll
          for (int i = 0; i < VP; ++i) x[i] = rv ? x[i] : 0.f;
        }
        reduce_scatter16<VP>(x, lane);
        float* row = sb + ((wv * CQ + qc) * 4 + r) * VP;
        if constexpr (VP >= 16) {
#pragma unroll
          for (int i = 0; i < VP / 16; ++i) row[(VP / 16) * n + i] = x[i];
        } else {
          if (n % (16 / VP) == 0) row[n / (16 / VP)] = x[0];
        }
      };
      if (q >= 16 && j0 + 4 <= m)   // (q >= nq implies j0 >= m: masked)
        quad(BoolTag<false>{});
      else
        quad(BoolTag<true>{});
    }
    }
    if (more) fill.store(afr + (buf ^ 1) * (CQ * 64 * 2 * NB), threadIdx.x, NTHR);
    // FP32 tiles of this chunk into the FP64 column sums
#pragma unroll
    for (int hh = 0; hh < HS; ++hh)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int v = 0; v < 4; ++v) col[hh][b][v] += (double)D[hh][b][v];
        D[hh][b] = f4{0.f, 0.f, 0.f, 0.f};
      }
    __syncthreads();  // the chunk is staged by every wavefront; the other buffer is free again
    // row partials of the chunk: the wavefronts' parts added in a fixed order
    for (int o = threadIdx.x; o < 4 * CQ * NBB; o += WAVES * 64) {
      const int e = o / (4 * CQ), rho = o - e * (4 * CQ);
      const int jj = 64 * s + 4 * q0 + rho;
      if (jj < m) {
        double re = 0.0, im = 0.0;
        for (int w = 0; w < WAVES; ++w) {
          const float* src = sb + (w * CQ * 4 + rho) * VP + 2 * e;
          re += (double)src[0];
          im += (double)src[1];
        }
        if constexpr (CPF > 1)
          rstg[e * Sh::ROWS + (ci % CPF) * 4 * CQ + rho] = cmk(re, im);
        else
          store_stream(rp + (int64_t)e * d.Tp + jj, cmk(re, im));
      }
    }
    if constexpr (CPF > 1) {
      if (ci % CPF == CPF - 1 || !more) {
        __syncthreads();
        const int base = 64 * s + 4 * q0 - (ci % CPF) * 4 * CQ;
        const int end = 64 * s + 4 * q0 + 4 * CQ;
        const int nrows = (end < m ? end : m) - base;
        for (int o = threadIdx.x; o < NBB * nrows; o += WAVES * 64) {
          const int e = o / nrows, row = o - e * nrows;
          store_stream(rp + (int64_t)e * d.Tp + base + row, rstg[e * Sh::ROWS + row]);
        }
        __syncthreads();
      }
    }
    buf ^= 1;
  }
  // column sums: high and low parts of each tile added in FP64 through LDS
  __syncthreads();  // every wavefront is done with the staging buffers
  double* fin = reinterpret_cast<double*>(smem) + (int64_t)wv * HS * NB * 256;
#pragma unroll
  for (int hh = 0; hh < HS; ++hh)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) fin[((hh * NB + b) * 16 + 4 * r + v) * 16 + n] = col[hh][b][v];
  __syncthreads();
  const int a = lane >> 4;
  if (a < NB && colv) {
#pragma unroll
    for (int hh = 0; hh < HS; ++hh)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const double* t = fin + (hh * NB + b) * 256;
        const int mre = 2 * a, mim = 2 * a + 1, lo = 2 * NB;
        double re = t[mre * 16 + n] + t[(lo + mre) * 16 + n];
        double im = t[mim * 16 + n] + t[(lo + mim) * 16 + n];
        const int c = (h0 + hh) * NBB + a * NB + b;
        colsum[rowbuf_idx(d, k, c, tp)] = cmk(re, im);
      }
  }
}

// ------------------------------------------------------------------ row assembly and update
// Thread per (k, t'), t' <= m.
//  EVAL/CORRECT, t' < m: I^{<,>}(t_m, t') = dt [bulk + end-point terms], where the
//   trapezoid corrections of the two integrals of eq. (CI) are
//     + 1/2 SR_mm G_{m t'} - 1/2 SR_m0 G_{0 t'}                                  (first, [0, t_m])
//     + [t' > 0] (-1/2 Sigma_{m t'} GR_{t' t'} + 1/2 Sigma_{m0} GR_{0 t'})       (second, [0, t'])
//   with GR = G^> - G^<, G_{0 t'} = -(G_{t' 0})^dag.
//  PREDICT/CORRECT/UPDATE, t' < m: G(t_m, t') = V G(t_{m-1}, t') + Phi Ibar(t') (UPDATE: the
//   corrector's update with I(t_m, t') read back from an EVAL launch's output).
//  PREDICT/CORRECT/UPDATE, t' = m: rho_m = V rho_{m-1} V^dag - dt Vh Dbar Vh^dag and the
//   equal-time block G^< = i rho_m, G^> = -i (1 - rho_m).
// G_{j t'} (both components) for the end corrections of output t' < m: the diagonal from the
// band copy; stored blocks j > t' from the ring of recent rows (row m: the current iterate) or
// the column copies (j < qp); blocks above the diagonal as -G_{t' j}^dag from the column copies
// (j < qp) or the band (t' - j < qp). Every node the corrections visit is one of these.
// Component sc (nb^2 entries) of the block G(t_j, t') an end-point correction needs, from the
// copies that hold it (as end_block, for one component).
template <int NB>
__device__ __forceinline__ void end_block1(const Dims& d, const cplx* __restrict__ row64, const cplx* __restrict__ colq,
                                           const cplx* __restrict__ band, int k, int m, int j, int tp, int sc,
                                           cplx* G) {
  constexpr int NBB = NB * NB;
  if (j == tp) {
#pragma unroll
    for (int e = 0; e < NBB; ++e) G[e] = band[band_idx(d, k, sc * NBB + e, tp, 0)];
  } else if (j > tp) {
    if (j > m - d.rring) {
#pragma unroll
      for (int e = 0; e < NBB; ++e) G[e] = row64[row64_idx(d, j, k, sc * NBB + e, tp)];
    } else {
#pragma unroll
      for (int e = 0; e < NBB; ++e) G[e] = colq[colq_idx(d, k, sc * NBB + e, j, tp)];
    }
  } else {
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        int cs = sc * NBB + b * NB + a;
        cplx v = j < d.qp ? colq[colq_idx(d, k, cs, tp, j)] : band[band_idx(d, k, cs, tp, tp - j)];
        G[a * NB + b] = cneg(cconj(v));
      }
  }
}
template <int NB>
__device__ __forceinline__ void end_block(const Dims& d, const cplx* __restrict__ row64, const cplx* __restrict__ colq,
                                          const cplx* __restrict__ band, int k, int m, int j, int tp, cplx* G) {
  constexpr int NBB = NB * NB, C = 2 * NBB;
  if (j == tp) {
#pragma unroll
    for (int c = 0; c < C; ++c) G[c] = band[band_idx(d, k, c, tp, 0)];
  } else if (j > tp) {
    if (j > m - d.rring) {
#pragma unroll
      for (int c = 0; c < C; ++c) G[c] = row64[row64_idx(d, j, k, c, tp)];
    } else {
#pragma unroll
      for (int c = 0; c < C; ++c) G[c] = colq[colq_idx(d, k, c, j, tp)];
    }
  } else {
#pragma unroll
    for (int sc = 0; sc < 2; ++sc)
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          int cs = sc * NBB + b * NB + a;
          cplx v = j < d.qp ? colq[colq_idx(d, k, cs, tp, j)] : band[band_idx(d, k, cs, tp, tp - j)];
          G[sc * NBB + a * NB + b] = cneg(cconj(v));
        }
  }
}

// Threads per (k, t') of the row kernel: one carrying both components G^<, G^> (nb <= 3), or at
// nb = 4 two, lanes 2i and 2i + 1 carrying G^< and G^> (the state of both, 32 complex numbers in
// each of several rows, would not fit one thread's registers).
template <int NB>
struct RowSplit {
  static constexpr int SCN = NB == 4 ? 1 : 2;   // components per thread
  static constexpr int TPT = 2 / SCN;           // threads per (k, t')
  static constexpr int TPB = 256 / TPT;         // t' per block of 256 threads
  // nb = 4: the strips' row partials are summed into slot 0 by k_rowpart_fold before the row
  // kernel runs (at one wave per SIMD, the row kernel's serial gather of up to n_t / 64 slots
  // would be latency-bound)
  static constexpr bool FOLD = NB == 4;
  // nb = 4: a corrector pass runs as EVAL (the collision row, stored) + UPDATE (the update from
  // the stored row), two waves per SIMD each without spills: the fused kernel holds 256 VGPRs +
  // 100 AGPRs, one wave per SIMD
  static constexpr bool CSPLIT = NB == 4;
};

// Row term of the history sums at nb = 4: the per-strip partials of row t' (slots 0 .. t' / 64)
// summed in slot order into slot 0, one thread per (k, entry, t'). Each slot-0 element is read
// and written by its own thread only, so the fold is in place; it runs once after each history
// pass, and the row kernels then read slot 0 alone. The sum has the order of the row kernels'
// own gather, so the result is the same.
template <int NB>
__global__ __launch_bounds__(256) void k_rowpart_fold(Dims d, cplx* __restrict__ rowpart, int m) {
  const int nblk = (m + 255) / 256;           // blocks per (k, entry)
  const int ke = blockIdx.x / nblk;           // k * nb^2 + entry
  const int tp = (blockIdx.x - ke * nblk) * 256 + threadIdx.x;
  const int k = ke / (NB * NB), e = ke - k * (NB * NB);
  if (tp >= m) return;
  const int nslot = (tp >> 6) / d.spb + 1;
  if (nslot == 1) return;
  const int64_t off = (int64_t)e * d.Tp + tp;
  cplx* p0 = rowpart + (int64_t)k * d.Smax * d.nbb * d.Tp + off;   // slot 0 of (k, e, t')
  const int64_t step = (int64_t)d.nbb * d.Tp;                         // one slot further
  cplx s = p0[0];
  int q = 1;
  for (; q + 4 <= nslot; q += 4) {
    cplx v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = p0[(q + u) * step];
#pragma unroll
    for (int u = 0; u < 4; ++u) s = cadd(s, v[u]);
  }
  for (; q < nslot; ++q) s = cadd(s, p0[q * step]);
  p0[0] = s;
}

template <int NB, int MODE, bool GREG>
__global__ __launch_bounds__(256) void k_row(Dims d, void* __restrict__ hist, cplx* __restrict__ row64,
                                             const cplx* __restrict__ sig, const cplx* __restrict__ colsum,
                                             const cplx* __restrict__ rowpart, cplx* __restrict__ col0,
                                             cplx* __restrict__ diag, const cplx* __restrict__ Iprev,
                                             cplx* __restrict__ Icur, const cplx* __restrict__ props,
                                             const cplx* __restrict__ rho_prev, cplx* __restrict__ rho_cur,
                                             const cplx* __restrict__ Dprev, const cplx* __restrict__ Dcur, int m,
                                             double dt, int commit, double* __restrict__ chg, QuadW Q) {
  constexpr int NBB = NB * NB;
  constexpr int SCN = RowSplit<NB>::SCN, TPT = RowSplit<NB>::TPT;
  constexpr bool UPD = MODE == KBE_ROW_UPDATE || MODE == KBE_ROW_UPDATE_CHG;   // I(t_m, .) stored
  constexpr bool CHG = MODE == KBE_ROW_CORRECT || MODE == KBE_ROW_UPDATE_CHG;  // change output
  const int k = blockIdx.y;
  const int tp = blockIdx.x * RowSplit<NB>::TPB + threadIdx.x / TPT;
  const int sc0 = SCN == 1 ? (threadIdx.x & 1) : 0;   // first component of this thread
  if (tp > m) return;   // (both lanes of a pair leave together)
  if (MODE == KBE_ROW_EVAL && tp == m) return;
  const cplx* P = props + (int64_t)k * 3 * NBB;
  double dmax = 0.0;
  if (tp < m) {
    cplx rs[NBB];   // row partials of the history sums, shared by both components (gathered after
                    // the first component's end-point terms, which need the registers more)
#pragma unroll
    for (int ls = 0; ls < SCN; ++ls) {
      const int sc = sc0 + ls;
      cplx In[NBB];
      if (MODE == KBE_ROW_CORRECT || MODE == KBE_ROW_EVAL) {
        // end-point terms of component sc, accumulated term by term
        cplx E[NBB];
        mat_zero<NB>(E);
        if constexpr (!GREG) {
          // trapezoid: half weights at j = 0 and j = m (first integral), j = 0 and j = t' (second)
          {
            cplx SRmm[NBB], Gm[NBB];
#pragma unroll
            for (int e = 0; e < NBB; ++e) {
              SRmm[e] = cscal(sig[sig_idx(d, k, 2, e, m)], 0.5);
              Gm[e] = row64[row64_idx(d, m, k, sc * NBB + e, tp)];
            }
            mm_acc<NB>(E, SRmm, Gm);
          }
          // G(t_0, t') of both components: G_00, or -G(t', t_0)^dag
          auto g0 = [&](int c, int a, int b) {
            return tp == 0 ? col0[colq_idx(d, k, c * NBB + a * NB + b, 0, 0)]
                           : cneg(cconj(col0[colq_idx(d, k, c * NBB + b * NB + a, tp, 0)]));
          };
          {
            cplx SRm0[NBB], G0[NBB];
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
              for (int b = 0; b < NB; ++b) {
                SRm0[a * NB + b] = cscal(sig[sig_idx(d, k, 2, a * NB + b, 0)], -0.5);
                G0[a * NB + b] = g0(sc, a, b);
              }
            mm_acc<NB>(E, SRm0, G0);
          }
          if (tp > 0) {
            cplx St[NBB], GRtt[NBB];
#pragma unroll
            for (int e = 0; e < NBB; ++e) {
              St[e] = cscal(sig[sig_idx(d, k, sc, e, tp)], -0.5);
              GRtt[e] = csub(diag[band_idx(d, k, NBB + e, tp, 0)], diag[band_idx(d, k, e, tp, 0)]);
            }
            mm_acc<NB>(E, St, GRtt);
            cplx S0[NBB], GR0t[NBB];
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
              for (int b = 0; b < NB; ++b) {
                S0[a * NB + b] = cscal(sig[sig_idx(d, k, sc, a * NB + b, 0)], 0.5);
                GR0t[a * NB + b] = csub(g0(1, a, b), g0(0, a, b));
              }
            mm_acc<NB>(E, S0, GR0t);
          }
        } else {
          // Gregory end corrections (d.qp nodes per end): against the bulk's unit weights,
          //   E = sum_j (w^(m)_j - [j < m]) SR_mj G_jt'  +  sum_{j <= t'} (w^(t')_j - [j < t']) Sigma_mj GA_jt',
          // nonzero on the nodes j < q' and j > N - q' of each interval (q' = min(qp, N + 1)).
          const int qm = d.qp < m + 1 ? d.qp : m + 1;
          for (int r = 0; r < 2; ++r) {
            int j0 = r == 0 ? 0 : (qm > m - qm + 1 ? qm : m - qm + 1);
            int j1 = r == 0 ? qm : m + 1;
            for (int j = j0; j < j1; ++j) {
              double w = quad_w(Q, j, m) - (j < m ? 1.0 : 0.0);
              if (w == 0.0) continue;
              cplx G[NBB], SR[NBB];
              end_block1<NB>(d, row64, col0, diag, k, m, j, tp, sc, G);
#pragma unroll
              for (int e = 0; e < NBB; ++e) SR[e] = cscal(sig[sig_idx(d, k, 2, e, j)], w);
              mm_acc<NB>(E, SR, G);
            }
          }
          if (tp > 0) {
            const int qt = d.qp < tp + 1 ? d.qp : tp + 1;
            for (int r = 0; r < 2; ++r) {
              int j0 = r == 0 ? 0 : (qt > tp - qt + 1 ? qt : tp - qt + 1);
              int j1 = r == 0 ? qt : tp + 1;
              for (int j = j0; j < j1; ++j) {
                double w = quad_w(Q, j, tp) - (j < tp ? 1.0 : 0.0);
                if (w == 0.0) continue;
                cplx GA[NBB], Gg[NBB], S[NBB];
                end_block1<NB>(d, row64, col0, diag, k, m, j, tp, 0, GA);
                end_block1<NB>(d, row64, col0, diag, k, m, j, tp, 1, Gg);
#pragma unroll
                for (int e = 0; e < NBB; ++e) {
                  GA[e] = csub(GA[e], Gg[e]);  // -(G^> - G^<)
                  S[e] = cscal(sig[sig_idx(d, k, sc, e, j)], w);
                }
                mm_acc<NB>(E, S, GA);
              }
            }
          }
        }
        if (ls == 0) {
          mat_zero<NB>(rs);
          const int nslot = RowSplit<NB>::FOLD ? 1 : (tp >> 6) / d.spb + 1;
          // slots in groups of 4: the loads of a group are issued together
          int q = 0;
          for (; q + 4 <= nslot; q += 4) {
            cplx v[4][NBB];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const cplx* rp = rowpart_slot(d, rowpart, k, q + u);
#pragma unroll
              for (int e = 0; e < NBB; ++e) v[u][e] = rp[(int64_t)e * d.Tp + tp];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
              for (int e = 0; e < NBB; ++e) rs[e] = cadd(rs[e], v[u][e]);
          }
          for (; q < nslot; ++q) {
            const cplx* rp = rowpart_slot(d, rowpart, k, q);
#pragma unroll
            for (int e = 0; e < NBB; ++e) rs[e] = cadd(rs[e], rp[(int64_t)e * d.Tp + tp]);
          }
        }
#pragma unroll
        for (int e = 0; e < NBB; ++e) {
          In[e] = cscal(cadd(cadd(colsum[rowbuf_idx(d, k, sc * NBB + e, tp)], rs[e]), E[e]), dt);
          Icur[rowbuf_idx(d, k, sc * NBB + e, tp)] = In[e];
        }
      }
      if (MODE != KBE_ROW_EVAL) {
        // G(t_m, t') = V G(t_{m-1}, t') + Phi Ibar(t') for component sc
        cplx Ib[NBB], Go[NBB], g[NBB];
#pragma unroll
        for (int e = 0; e < NBB; ++e) {
          cplx ip = Iprev[rowbuf_idx(d, k, sc * NBB + e, tp)];
          if constexpr (UPD) In[e] = Icur[rowbuf_idx(d, k, sc * NBB + e, tp)];
          Ib[e] = (MODE == KBE_ROW_PREDICT) ? ip : cscal(cadd(ip, In[e]), 0.5);
          Go[e] = row64[row64_idx(d, m - 1, k, sc * NBB + e, tp)];
        }
        mat_zero<NB>(g);
        {
          cplx V[NBB];
#pragma unroll
          for (int e = 0; e < NBB; ++e) V[e] = P[e];
          mm_acc<NB>(g, V, Go);
        }
        {
          cplx Phi[NBB];
#pragma unroll
          for (int e = 0; e < NBB; ++e) Phi[e] = P[2 * NBB + e];
          mm_acc<NB>(g, Phi, Ib);
        }
#pragma unroll
        for (int e = 0; e < NBB; ++e) {
          const int c = sc * NBB + e;
          if (CHG && chg) {  // change against the iterate this pass started from
            cplx dg = csub(g[e], row64[row64_idx(d, m, k, c, tp)]);
            dmax = fmax(dmax, sqrt(dg.x * dg.x + dg.y * dg.y));
          }
          row64[row64_idx(d, m, k, c, tp)] = g[e];
          if (commit) {
            commit_store(d, hist, k, c, m, tp, g[e]);
            if (tp < d.qp) col0[colq_idx(d, k, c, m, tp)] = g[e];
            if (m - tp < d.qp) diag[band_idx(d, k, c, m, m - tp)] = g[e];
          }
        }
      }
    }
  } else if (sc0 == 0) {
    // tp == m, PREDICT or CORRECT: density matrix and equal-time block (one thread per k)
    cplx V[NBB], Vh[NBB], r0[NBB], Db[NBB], t1[NBB], rho[NBB], t2[NBB];
#pragma unroll
    for (int e = 0; e < NBB; ++e) {
      V[e] = P[e];
      Vh[e] = P[NBB + e];
      r0[e] = rho_prev[(int64_t)k * NBB + e];
      cplx dp = Dprev[(int64_t)k * NBB + e];
      Db[e] = (MODE == KBE_ROW_PREDICT) ? dp : cscal(cadd(dp, Dcur[(int64_t)k * NBB + e]), 0.5);
    }
    mat_zero<NB>(t1);
    mm_acc<NB>(t1, V, r0);
    mat_zero<NB>(rho);
    mm_acc_bdag<NB>(rho, t1, V);
    mat_zero<NB>(t1);
    mm_acc<NB>(t1, Vh, Db);
    mat_zero<NB>(t2);
    mm_acc_bdag<NB>(t2, t1, Vh);
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        int e = a * NB + b;
        cplx rv = csub(rho[e], cscal(t2[e], dt));
        rho_cur[(int64_t)k * NBB + e] = rv;
        cplx gg[2];
        gg[0] = cmuli(rv);
        gg[1] = cneg(cmuli(csub(cmk(a == b ? 1.0 : 0.0, 0.0), rv)));
#pragma unroll
        for (int sc = 0; sc < 2; ++sc) {
          int c = sc * NBB + e;
          if (CHG && chg) {
            cplx dg = csub(gg[sc], row64[row64_idx(d, m, k, c, m)]);
            dmax = fmax(dmax, sqrt(dg.x * dg.x + dg.y * dg.y));
          }
          row64[row64_idx(d, m, k, c, m)] = gg[sc];
          if (commit) {
            commit_store(d, hist, k, c, m, m, gg[sc]);
            diag[band_idx(d, k, c, m, 0)] = gg[sc];
            if (m < d.qp) col0[colq_idx(d, k, c, m, m)] = gg[sc];
          }
        }
      }
  }
  if (CHG && chg) {
    if constexpr (TPT == 2) dmax = fmax(dmax, __shfl_xor(dmax, 1));   // the pair's two components
    if (sc0 == 0) chg[(int64_t)k * d.Tp + tp] = dmax;
  }
}

// Largest change of the corrector's row: out[0] = max over k and t' <= m of chg[k][t'].
// One block, a fixed reduction order (max is exact, so any order gives the same value).
__global__ __launch_bounds__(1024) void k_change_max(const double* __restrict__ chg, int nk, int Tp, int m,
                                                     double* __restrict__ out) {
  __shared__ double red[1024];
  double mx = 0.0;
  for (int k = 0; k < nk; ++k)
    for (int t = threadIdx.x; t <= m; t += 1024) mx = fmax(mx, chg[(int64_t)k * Tp + t]);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// ------------------------------------------------------------------ dipole kick
// The kick of the dipole pulse of eq. (dipole) on the completed slice m: G(t_m, t') <- K G(t_m, t')
// for t' < m and K G K^dag on the equal-time block (both components), rho_m <- K rho_m K^dag,
// K = kc 1 - i ks X (X: ones between bands 0 and 1; nb = 2). Thread per (k, t'); the FP64
// working copy of the row is the source, and every copy of the row is rewritten (packed
// history, working copy, column and diagonal copies). rho goes to rhoX and rhoY (both density
// buffers at t = 0).
template <int NB>
__global__ __launch_bounds__(256) void k_kick_row(Dims d, void* __restrict__ hist, cplx* __restrict__ row64,
                                                  cplx* __restrict__ col0, cplx* __restrict__ diag, cplx* rhoX,
                                                  cplx* rhoY, int m, double kc, double ks) {
  static_assert(NB == 2, "the dipole kick couples the two bands of the paper's model");
  int k = blockIdx.y;
  int tp = blockIdx.x * 256 + threadIdx.x;
  if (tp > m) return;
  // (K G)_ab = kc G_ab - i ks G_{1-a, b};  (T K^dag)_ab = kc T_ab + i ks T_{a, 1-b}
  auto kick = [&](const cplx* G, cplx* out, bool both_sides) {
    cplx T[4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) T[a * 2 + b] = csub(cscal(G[a * 2 + b], kc), cmuli(cscal(G[(1 - a) * 2 + b], ks)));
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        out[a * 2 + b] = both_sides ? cadd(cscal(T[a * 2 + b], kc), cmuli(cscal(T[a * 2 + 1 - b], ks))) : T[a * 2 + b];
  };
#pragma unroll
  for (int sc = 0; sc < 2; ++sc) {
    cplx G[4], R[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) G[e] = row64[row64_idx(d, m, k, sc * 4 + e, tp)];
    kick(G, R, tp == m);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int c = sc * 4 + e;
      row64[row64_idx(d, m, k, c, tp)] = R[e];
      commit_store(d, hist, k, c, m, tp, R[e]);
      if (tp < d.qp) col0[colq_idx(d, k, c, m, tp)] = R[e];
      if (m - tp < d.qp) diag[band_idx(d, k, c, m, m - tp)] = R[e];
    }
  }
  if (tp == m) {
    cplx r[4], R[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) r[e] = rhoX[(int64_t)k * 4 + e];
    kick(r, R, true);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      rhoX[(int64_t)k * 4 + e] = R[e];
      rhoY[(int64_t)k * 4 + e] = R[e];
    }
  }
}

// ------------------------------------------------------------------ observables
template <int NB>
__global__ __launch_bounds__(256) void k_obs(Dims d, const cplx* __restrict__ hop, const cplx* __restrict__ rho,
                                             const cplx* __restrict__ Icur, int m, double t, double A,
                                             double Ax, double Ay, int interaction, int hf, double U,
                                             double spin, double* __restrict__ obs) {
  constexpr int NBB = NB * NB;
  constexpr int NV = 6 + 2 * NB;  // N, Ekin, Ehf, Ecorr, Jx, Jy, n_orb[NB], n_band[NB]
  __shared__ double red[NV][256];
  __shared__ cplx loc_s[NBB];
  int tid = threadIdx.x;
  // local density matrix for the mean field
  {
    __shared__ cplx lds[NBB * 256];
    cplx loc[NBB];
#pragma unroll
    for (int e = 0; e < NBB; ++e) loc[e] = czero();
    for (int k = tid; k < d.nk; k += 256)
#pragma unroll
      for (int e = 0; e < NBB; ++e) loc[e] = cadd(loc[e], rho[(int64_t)k * NBB + e]);
    block_sum_cplx<NBB>(loc, lds);
    if (tid == 0)
#pragma unroll
      for (int e = 0; e < NBB; ++e) loc_s[e] = cscal(loc[e], 1.0 / d.nk);
    __syncthreads();
  }
  cplx hfm[NBB], ob[NBB];
#pragma unroll
  for (int e = 0; e < NBB; ++e) {
    hfm[e] = czero();
    ob[e] = czero();
  }
  if (interaction == KBE_DEV_INT_HUBBARD) {
    if (hf)
#pragma unroll
      for (int a = 0; a < NB; ++a) hfm[a * NB + a] = cmk(U * loc_s[a * NB + a].x, 0.0);
  } else {
    if constexpr (NB == 2) {
      ob[3] = cmk(-U, 0.0);
      if (hf) {
        hfm[0] = cmk(U * loc_s[3].x, 0.0);
        hfm[3] = cmk(U * loc_s[0].x, 0.0);
        hfm[1] = cscal(loc_s[1], -U);
        hfm[2] = cscal(loc_s[2], -U);
      }
    }
  }
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  for (int k = tid; k < d.nk; k += 256) {
    cplx r[NBB], h[NBB], v[NBB], Vv[NBB];
    double w[NB];
#pragma unroll
    for (int e = 0; e < NBB; ++e) r[e] = rho[(int64_t)k * NBB + e];
    bloch_h0<NB>(hop, d.nkx, d.nky, k, Ax, Ay, h);
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      acc[0] += r[a * NB + a].x;
      acc[6 + a] += r[a * NB + a].x;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        acc[1] += cmul(cadd(h[a * NB + b], ob[a * NB + b]), r[b * NB + a]).x;
        acc[2] += cmul(hfm[a * NB + b], r[b * NB + a]).x;
      }
      acc[3] += 0.5 * Icur[rowbuf_idx(d, k, a * NB + a, m)].y;  // Re(-i/2 I) = Im(I)/2
    }
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
      bloch_vel<NB>(hop, d.nkx, d.nky, k, Ax, Ay, dir, v);
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[4 + dir] += cmul(v[a * NB + b], r[b * NB + a]).x;
    }
    jacobi_eigh<NB>(h, w, Vv);
#pragma unroll
    for (int bnd = 0; bnd < NB; ++bnd) {
      double sacc = 0.0;
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
          sacc += cmul(cmul(cconj(Vv[a * NB + bnd]), r[a * NB + b]), Vv[b * NB + bnd]).x;
      acc[6 + NB + bnd] += sacc;
    }
  }
#pragma unroll
  for (int i = 0; i < NV; ++i) red[i][tid] = acc[i];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s)
#pragma unroll
      for (int i = 0; i < NV; ++i) red[i][tid] += red[i][tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    double inv = 1.0 / d.nk;
    double* o = obs + (int64_t)m * KBE_DEV_NOBS;
    for (int i = 0; i < KBE_DEV_NOBS; ++i) o[i] = 0.0;
    o[0] = t;
    o[1] = spin * red[0][0] * inv;
    o[2] = spin * red[1][0] * inv;
    o[3] = 0.5 * spin * red[2][0] * inv;
    o[4] = spin * red[3][0] * inv;
    o[5] = o[2] + o[3] + o[4];
    o[6] = spin * red[4][0] * inv;
    o[7] = spin * red[5][0] * inv;
    o[8] = A;
    for (int a = 0; a < NB; ++a) o[9 + a] = red[6 + a][0] * inv;
    for (int b = 0; b < NB; ++b) o[13 + b] = red[6 + NB + b][0] * inv;
  }
}

// ------------------------------------------------------------------ aux copies
// Refresh the FP64 working copies from history rows 0..m: columns 0..qp-1, the diagonal band
// of width qp, and the ring of the last rring rows (m - rring + 1 .. m).
template <int NB>
__global__ void k_aux(Dims d, const void* __restrict__ hist, cplx* __restrict__ row64, cplx* __restrict__ col0,
                      cplx* __restrict__ diag, int m) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int kc = blockIdx.y;
  if (j > m) return;
  int k = kc / d.C, c = kc - (kc / d.C) * d.C;
  for (int q = 0; q < d.qp && q <= j; ++q) {
    col0[colq_idx(d, k, c, j, q)] = history_load(d, hist, k, c, j, q);
    diag[band_idx(d, k, c, j, q)] = history_load(d, hist, k, c, j, j - q);
  }
  for (int r = m; r >= 0 && r > m - d.rring; --r)
    if (j <= r) row64[row64_idx(d, r, k, c, j)] = history_load(d, hist, k, c, r, j);
}

// ------------------------------------------------------------------ launchers
// Dynamic LDS above 64 KB (the self-energy tile of a long chain: 82 KB at N_k = 1024) is asked
// for explicitly; gfx950 gives a workgroup up to 160 KB.
static hipError_t allow_lds(const void* kern, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int NB>
struct Launch {
  static hipError_t init(const Dims& d, const LaunchArgs& a, hipStream_t st) {
    int nb64 = (d.nk + 63) / 64;
    hipLaunchKernelGGL(k_init_eig<NB>, dim3(nb64), dim3(64), 0, st, d, a.hop, a.Ax, a.Ay, a.eig_w, a.eig_U);
    hipLaunchKernelGGL(k_init_mu, dim3(1), dim3(256), 0, st, d.nk * NB, (const double*)a.eig_w, a.temp,
                       a.target, a.mu);
    hipLaunchKernelGGL(k_init_rho<NB>, dim3(nb64), dim3(64), 0, st, d, (const double*)a.eig_w,
                       (const cplx*)a.eig_U, (const double*)a.mu, a.temp, a.rho_prev, a.rho_cur, a.hist,
                       a.row64, a.col0, a.diag);
    return hipGetLastError();
  }
  static hipError_t hf(const Dims& d, const LaunchArgs& a, double wb, hipStream_t st) {
    hipLaunchKernelGGL(k_hf<NB>, dim3(1), dim3(256), 0, st, d, (const cplx*)a.rho_prev, (const cplx*)a.rho_cur,
                       wb, a.interaction, a.hf, a.U, a.hfbuf);
    return hipGetLastError();
  }
  static hipError_t props(const Dims& d, const LaunchArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_props<NB>, dim3((d.nk + 3) / 4), dim3(256), 0, st, d, a.hop, (const cplx*)a.hfbuf,
                       a.Ax, a.Ay, a.dt, a.props);
    return hipGetLastError();
  }
  static hipError_t sigma(const Dims& d, const LaunchArgs& a, int m, hipStream_t st) {
    int total = (m + 1) * NB * NB;
    int per = (total + 7) / 8;
    size_t shm = (size_t)(4 * d.nk + d.nkx + d.nky) * sizeof(cplx);
    if constexpr (NB == 2) {
      if (a.interaction == KBE_DEV_INT_INTERBAND) {
        auto fwd = k_sigma_fwd<0, 0>;
        auto ib = k_sigma_ib<0, 0>;
        if (d.nkx == 16 && d.nky == 1) {
          fwd = k_sigma_fwd<16, 1>;
          ib = k_sigma_ib<16, 1>;
        }
        hipError_t e = allow_lds((const void*)fwd, shm);
        if (e == hipSuccess) e = allow_lds((const void*)ib, shm);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(fwd, dim3(per * 8), dim3(256), shm, st, d, (const cplx*)a.row64, a.gR, m);
        hipLaunchKernelGGL(ib, dim3(per * 8), dim3(256), shm, st, d, (const cplx*)a.gR, a.sig, m, a.UU, a.corr);
        return hipGetLastError();
      }
    }
    // grids of the standard workloads with compile-time transforms, any other grid at run time
    auto kern = k_sigma<NB, 0, 0>;
    if (d.nkx == 24 && d.nky == 24) kern = k_sigma<NB, 24, 24>;
    else if (d.nkx == 16 && d.nky == 16) kern = k_sigma<NB, 16, 16>;
    else if (d.nkx == 12 && d.nky == 12) kern = k_sigma<NB, 12, 12>;
    else if (d.nkx == 16 && d.nky == 1) kern = k_sigma<NB, 16, 1>;
    hipError_t e = allow_lds((const void*)kern, shm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(per * 8), dim3(256), shm, st, d, (const cplx*)a.row64, a.sig, m, a.UU, a.corr);
    return hipGetLastError();
  }
  static hipError_t diag_I(const Dims& d, const LaunchArgs& a, int m, hipStream_t st) {
    hipLaunchKernelGGL(k_diag_I<NB>, dim3(d.nk), dim3(256), 0, st, d, (const cplx*)a.row64, (const cplx*)a.sig,
                       a.I_cur, a.D_cur, m, a.dt, a.quad);
    return hipGetLastError();
  }
  static hipError_t bulk(const Dims& d, const LaunchArgs& a, int m, hipStream_t st) {
    if (m < 1) return hipSuccess;
    int ns = (m + 63) / 64;
    if (d.mfma) {
      hipLaunchKernelGGL(k_hist_mfma<NB>, dim3(ns * d.nk), dim3(MfmaShape<NB>::WAVES * 64), 0, st, d,
                         (const float2*)a.hist, (const cplx*)a.sig, a.colsum, a.rowpart, m);
      return hipGetLastError();
    }
    if constexpr (NB <= 2) {
      int np = (ns + 1) / 2;  // pairs of strips
      if (d.fp32)
        hipLaunchKernelGGL(k_hist_pair32<NB>, dim3(np * d.nk), dim3(256), 0, st, d, (const cplx32*)a.hist,
                           (const cplx*)a.sig, a.colsum, a.rowpart, m);
      else
        hipLaunchKernelGGL(k_hist_pair<NB>, dim3(np * d.nk), dim3(256), 0, st, d, (const cplx*)a.hist,
                           (const cplx*)a.sig, a.colsum, a.rowpart, m);
    } else if constexpr (NB == 4) {
      if (d.fp32)
        hipLaunchKernelGGL(k_hist_bulk32_split<NB>, dim3(ns * d.nk), dim3(256), 0, st, d, (const cplx32*)a.hist,
                           (const cplx*)a.sig, a.colsum, a.rowpart, m);
      else
        hipLaunchKernelGGL(k_hist_bulk_split<NB>, dim3(ns * d.nk), dim3(256), 0, st, d, (const cplx*)a.hist,
                           (const cplx*)a.sig, a.colsum, a.rowpart, m);
    } else {
      if (d.fp32)
        hipLaunchKernelGGL(k_hist_bulk32<NB>, dim3(ns * d.nk), dim3(256), 0, st, d, (const cplx32*)a.hist,
                           (const cplx*)a.sig, a.colsum, a.rowpart, m);
      else
        hipLaunchKernelGGL(k_hist_bulk<NB>, dim3(ns * d.nk), dim3(256), 0, st, d, (const cplx*)a.hist,
                           (const cplx*)a.sig, a.colsum, a.rowpart, m);
    }
    return hipGetLastError();
  }
  static hipError_t fold(const Dims& d, const LaunchArgs& a, int m, hipStream_t st) {
    if constexpr (RowSplit<NB>::FOLD) {
      if (m < 65) return hipSuccess;   // one strip: nothing to fold
      hipLaunchKernelGGL(k_rowpart_fold<NB>, dim3((m + 255) / 256 * NB * NB * d.nk), dim3(256), 0, st, d,
                         a.rowpart, m);
      return hipGetLastError();
    }
    return hipSuccess;
  }
  static hipError_t row(const Dims& d, const LaunchArgs& a, int m, int mode, hipStream_t st) {
    dim3 grid((m + 1 + RowSplit<NB>::TPB - 1) / RowSplit<NB>::TPB, d.nk);
#define KBE_ROW_ARGS                                                                                      \
  d, a.hist, a.row64, (const cplx*)a.sig, (const cplx*)a.colsum, (const cplx*)a.rowpart, a.col0, a.diag, \
      (const cplx*)a.I_prev, a.I_cur, (const cplx*)a.props, (const cplx*)a.rho_prev, a.rho_cur,           \
      (const cplx*)a.D_prev, (const cplx*)a.D_cur, m, a.dt, a.commit, a.chg, a.quad
    // the trapezoid's end terms are a fixed handful; Gregory corrections loop over their nodes
    if (d.qp > 1) {
      if (mode == KBE_ROW_PREDICT)
        hipLaunchKernelGGL((k_row<NB, KBE_ROW_PREDICT, true>), grid, dim3(256), 0, st, KBE_ROW_ARGS);
      else if (mode == KBE_ROW_CORRECT && !RowSplit<NB>::CSPLIT)
        hipLaunchKernelGGL((k_row<NB, KBE_ROW_CORRECT, true>), grid, dim3(256), 0, st, KBE_ROW_ARGS);
      else
        hipLaunchKernelGGL((k_row<NB, KBE_ROW_EVAL, true>), grid, dim3(256), 0, st, KBE_ROW_ARGS);
    } else {
      if (mode == KBE_ROW_PREDICT)
        hipLaunchKernelGGL((k_row<NB, KBE_ROW_PREDICT, false>), grid, dim3(256), 0, st, KBE_ROW_ARGS);
      else if (mode == KBE_ROW_CORRECT && !RowSplit<NB>::CSPLIT)
        hipLaunchKernelGGL((k_row<NB, KBE_ROW_CORRECT, false>), grid, dim3(256), 0, st, KBE_ROW_ARGS);
      else
        hipLaunchKernelGGL((k_row<NB, KBE_ROW_EVAL, false>), grid, dim3(256), 0, st, KBE_ROW_ARGS);
    }
    if (mode == KBE_ROW_CORRECT && RowSplit<NB>::CSPLIT) {
      if (a.chg)
        hipLaunchKernelGGL((k_row<NB, KBE_ROW_UPDATE_CHG, false>), grid, dim3(256), 0, st, KBE_ROW_ARGS);
      else
        hipLaunchKernelGGL((k_row<NB, KBE_ROW_UPDATE, false>), grid, dim3(256), 0, st, KBE_ROW_ARGS);
    }
#undef KBE_ROW_ARGS
    return hipGetLastError();
  }
  static hipError_t obs(const Dims& d, const LaunchArgs& a, int m, double t, double A, hipStream_t st) {
    hipLaunchKernelGGL(k_obs<NB>, dim3(1), dim3(256), 0, st, d, a.hop, (const cplx*)a.rho_cur,
                       (const cplx*)a.I_cur, m, t, A, a.Ax, a.Ay, a.interaction, a.hf, a.U, a.spin, a.obs);
    return hipGetLastError();
  }
  static hipError_t aux(const Dims& d, const LaunchArgs& a, int m, hipStream_t st) {
    dim3 grid((m + 1 + 255) / 256, d.nk * d.C);
    hipLaunchKernelGGL(k_aux<NB>, grid, dim3(256), 0, st, d, (const void*)a.hist, a.row64, a.col0, a.diag, m);
    return hipGetLastError();
  }
};

hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

#define KBE_DISPATCH(NBV, CALL)                     \
  switch (NBV) {                                    \
    case 1: return Launch<1>::CALL;                 \
    case 2: return Launch<2>::CALL;                 \
    case 3: return Launch<3>::CALL;                 \
    case 4: return Launch<4>::CALL;                 \
    default: return hipErrorInvalidValue;           \
  }

hipError_t launch_init(const Dims& d, const LaunchArgs& a, hipStream_t st) { KBE_DISPATCH(d.nb, init(d, a, st)); }
hipError_t launch_hf(const Dims& d, const LaunchArgs& a, double wb, hipStream_t st) {
  KBE_DISPATCH(d.nb, hf(d, a, wb, st));
}
hipError_t launch_props(const Dims& d, const LaunchArgs& a, hipStream_t st) { KBE_DISPATCH(d.nb, props(d, a, st)); }
hipError_t launch_sigma(const Dims& d, const LaunchArgs& a, int m, hipStream_t st) {
  KBE_DISPATCH(d.nb, sigma(d, a, m, st));
}
hipError_t launch_kick(const Dims& d, const LaunchArgs& a, int m, double kc, double ks, cplx* rho_other,
                       hipStream_t st) {
  if (d.nb != 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_kick_row<2>, dim3((m + 1 + 255) / 256, d.nk), dim3(256), 0, st, d, a.hist, a.row64, a.col0,
                     a.diag, a.rho_cur, rho_other, m, kc, ks);
  return hipGetLastError();
}
hipError_t launch_sigma_direct(const Dims& d, const LaunchArgs& a, int m, hipStream_t st) {
  size_t shm = (size_t)(6 * d.nk + d.nk / 8) * sizeof(cplx);
  hipError_t e = allow_lds((const void*)k_sigma_direct, shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sigma_direct, dim3((m + 1) * 4), dim3(512), shm, st, d, (const cplx*)a.row64, a.sig, m, a.UU,
                     a.corr);
  return hipGetLastError();
}
hipError_t launch_diag_I(const Dims& d, const LaunchArgs& a, int m, hipStream_t st) {
  KBE_DISPATCH(d.nb, diag_I(d, a, m, st));
}
hipError_t launch_bulk(const Dims& d, const LaunchArgs& a, int m, hipStream_t st) {
  KBE_DISPATCH(d.nb, bulk(d, a, m, st));
}
hipError_t launch_rowpart_fold(const Dims& d, const LaunchArgs& a, int m, hipStream_t st) {
  KBE_DISPATCH(d.nb, fold(d, a, m, st));
}
hipError_t launch_row(const Dims& d, const LaunchArgs& a, int m, int mode, hipStream_t st) {
  KBE_DISPATCH(d.nb, row(d, a, m, mode, st));
}
hipError_t launch_change_max(const Dims& d, const double* chg, int m, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_change_max, dim3(1), dim3(1024), 0, st, chg, d.nk, d.Tp, m, out);
  return hipGetLastError();
}
hipError_t launch_obs(const Dims& d, const LaunchArgs& a, int m, double t, double A, hipStream_t st) {
  KBE_DISPATCH(d.nb, obs(d, a, m, t, A, st));
}
hipError_t launch_aux(const Dims& d, const LaunchArgs& a, int m, hipStream_t st) {
  KBE_DISPATCH(d.nb, aux(d, a, m, st));
}

}  // namespace kbe
