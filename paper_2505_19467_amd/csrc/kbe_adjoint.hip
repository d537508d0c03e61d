// Adjoint (reverse-mode) kernels of the Kadanoff-Baym propagation step (gfx950).
//
// The reverse sweep runs the steps of Algorithm "prop" backwards. For a real loss L every
// complex quantity x carries an adjoint xbar = dL/dRe(x) + i dL/dIm(x), with the rules
//   y = A x        -> xbar += A^dag ybar,     Abar += ybar x^dag
//   y = A B^dag    -> Abar += ybar B,         Bbar += ybar^dag A
//   y = conj(x)    -> xbar += conj(ybar)
// and for a real parameter p:  dL/dp += Re sum conj(ybar) dy/dp.
//
//   k_adj_bulk    adjoint of the history sums: reads the stored block, accumulates the
//                 self-energy adjoints (column sums in registers, row sums across lanes); in
//                 its fused form it also updates the adjoint history (read-modify-write, same
//                 strip-major layout) for both collision passes of a reverse step
//   k_adj_row     adjoint of the end-point and equal-time terms of eq. (CI): completes the
//                 self-energy adjoint row and the adjoint of the current row
//   k_adj_sigma   adjoint of eq. (2BSE) through the k <-> R transforms (Wirtinger products)
//   k_adj_update  adjoint of the predictor/corrector update of G(t_m, .) and rho_m
//   k_adj_props   adjoint of V, Vh, Phi: Frechet derivative of the augmented exponential
//   k_adj_hf      adjoint of the mean field and of the pulse; parameter gradients
//   k_adj_seed    adjoint of the final-time observable
//   k_adj_rho     rho_m = -i G^<(t_m, t_m) read back from the stored history diagonal
#include "kbe_adjoint.hpp"
#include "kbe_device.hpp"
#include "kbe_kernels.hpp"

namespace kbe {

// (A^dag B)_ij = sum_l conj(A_li) B_lj
template <int NB>
__device__ __forceinline__ void mm_acc_adag(cplx* acc, const cplx* A, const cplx* B) {
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int l = 0; l < NB; ++l) {
        cplx a = cconj(A[l * NB + i]);
        cmac(acc[i * NB + j], a, B[l * NB + j]);
      }
}

// ------------------------------------------------------------------ adjoint history sums
// Forward (weight 1, times dt), per stored block (j, t'), t' <= j <= m-1:
//   I^s(t') += dt SR_j G^s_{jt'};   t' < j:  I^<(j), I^>(j) += dt [-S^>_{t'} G^<_{jt'}^dag + S^<_{t'} G^>_{jt'}^dag]
// Adjoint with Ibar^s(t') and Irow(j) = Ibar^<(j) + Ibar^>(j):
//   lam^s_{jt'} += dt SR_j^dag Ibar^s(t');   t' < j:  lam^< -= dt Irow(j)^dag S^>_{t'}, lam^> += dt Irow(j)^dag S^<_{t'}
//   SRbar_j     += dt sum_{t'} sum_s Ibar^s(t') G^s_{jt'}^dag           (across lanes, per strip)
//   Sbar^>_{t'} -= dt sum_{j > t'} Irow(j) G^<_{jt'},  Sbar^<_{t'} += dt sum_{j > t'} Irow(j) G^>_{jt'}   (in lane)
// The lam terms are linear in (SR, Ibar, Irow, S): a reverse step's first pass (ADJ_SUMS) only
// reads the history for its Sigma adjoints, and its second pass (ADJ_FUSED) applies the lam
// terms of both passes in one read-modify-write of the adjoint history (the first pass's Sigma
// row and Ibar come in as sig1, Ibar1; their columns sit in LDS): 4 streams per reverse step
// instead of 6. Layout of the work as in the forward history sums: block = (strip s, k); lane l
// owns column 64 s + l (its Sigma, Ibar and Sigma-adjoint column sums in registers); in the
// fused pass each wavefront takes 16 consecutive rows of every 64-row chunk, in the read-only
// pass rows w, w + 4, ..., w + 60 (wavefront w), one row per iteration (the history block and,
// fused, the adjoint-history block of the row: 2 C 1 KB-contiguous loads in flight, then C 1 KB
// stores).
// The SRbar row partial of a row (nb^2 components) goes through one 64-lane reduce-scatter with
// the components as groups; the row partials of four 64-row chunks are staged in LDS and stored
// by the whole block as 4 KB runs per component. Rows past the strip's first 64 (and below m) run
// without bounds selects.
template <int NB, int MODE>
__global__ __launch_bounds__(256) void k_adj_bulk(Dims d, const cplx* __restrict__ hist, cplx* __restrict__ lam,
                                                  const cplx* __restrict__ sig, const cplx* __restrict__ Ibar,
                                                  const cplx* __restrict__ sig1, const cplx* __restrict__ Ibar1,
                                                  cplx* __restrict__ sbar_col, cplx* __restrict__ sbar_rowpart,
                                                  int m, double dt) {
  constexpr int NBB = NB * NB, C = 2 * NBB;
  constexpr int CH = (C < 8) ? C : 8;
  __shared__ cplx red[3][CH][64];
  constexpr int ROWS_ST = 256;   // row partials of four 64-row chunks, stored by the block at once
  __shared__ cplx stg[NBB][ROWS_ST];
  const int s = blockIdx.x / d.nk;
  const int k = blockIdx.x - s * d.nk;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // rows wavefront-uniform
  const int tp = 64 * s + lane;
  const bool colv = tp < m;
  const cplx* sk = sig + (int64_t)k * 3 * NBB * d.Tp;
  cplx Sl[NBB], Sg[NBB], Ib[C];
#pragma unroll
  for (int e = 0; e < NBB; ++e) {
    Sl[e] = colv ? sk[(0 * NBB + e) * d.Tp + tp] : czero();
    Sg[e] = colv ? sk[(1 * NBB + e) * d.Tp + tp] : czero();
  }
#pragma unroll
  for (int c = 0; c < C; ++c) Ib[c] = colv ? Ibar[rowbuf_idx(d, k, c, tp)] : czero();
  // ADJ_FUSED: the earlier pass's Sigma^<, Sigma^> and Ibar columns of the strip, in LDS
  __shared__ cplx xS[MODE == ADJ_FUSED ? 2 * NBB * 64 : 1];
  __shared__ cplx xI[MODE == ADJ_FUSED ? C * 64 : 1];
  const cplx* sk1 = sig1 + (int64_t)k * 3 * NBB * d.Tp;
  if constexpr (MODE == ADJ_FUSED) {
    for (int q = threadIdx.x; q < 2 * NBB * 64; q += 256) {
      const int l = q & 63, t = 64 * s + l;
      xS[q] = t < m ? sk1[(q >> 6) * d.Tp + t] : czero();
    }
    for (int q = threadIdx.x; q < C * 64; q += 256) {
      const int l = q & 63, t = 64 * s + l;
      xI[q] = t < m ? Ibar1[rowbuf_idx(d, k, q >> 6, t)] : czero();
    }
    __syncthreads();
  }
  cplx acc[C];  // [0, NBB): Sbar^<_{t'}, [NBB, C): Sbar^>_{t'}
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = czero();
  const int64_t base = strip_lane_base(d, k, s, lane);
  const cplx* hk = hist + base;
  cplx* lk = lam + base;
  cplx* rp = sbar_rowpart + ((int64_t)k * d.Smax + s) * NBB * d.Tp;
  for (int cb = 64 * s; cb < m; cb += 64) {
    // the read-only pass: wavefront w takes rows w, w + 4, ..., w + 60 (a chunk cut short by m
    // keeps all four busy); the fused pass: 16 consecutive rows (its read-modify-write stream
    // runs better in 128 KB runs per wavefront)
    constexpr int RS = MODE == ADJ_SUMS ? 4 : 1;
    const int rb = cb + (MODE == ADJ_SUMS ? wv : 16 * wv);
    const int cslot = ((cb - 64 * s) >> 6) % (ROWS_ST / 64);
    cplx* st = &stg[0][64 * cslot];   // st[e * ROWS_ST + (row - cb)]
    for (int i = 0; i < 16; ++i) {
      const int j = rb + RS * i;
      if (j >= m) break;
      auto row = [&](auto tag) {
        constexpr bool MASKED = decltype(tag)::value;
        const bool v = MASKED ? (colv && tp <= j) : true;
        const int64_t off = 64 * (int64_t)C * j;
        cplx G[C], L[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          G[c] = v ? load_stream(hk + off + 64 * c) : czero();
          if constexpr (MODE != ADJ_SUMS) L[c] = v ? load_stream(lk + off + 64 * c) : czero();
        }
        cplx SR[NBB], Irow[NBB];
#pragma unroll
        for (int e = 0; e < NBB; ++e) {
          SR[e] = sk[(2 * NBB + e) * d.Tp + j];
          Irow[e] = cadd(Ibar[rowbuf_idx(d, k, e, j)], Ibar[rowbuf_idx(d, k, NBB + e, j)]);
        }
        const bool rv = MASKED ? tp < j : true;
        if constexpr (MODE == ADJ_FUSED) {
          // adjoint history, accumulated into the loaded block with dt-scaled row factors:
          //   lam^s += (dt SR)^dag Ibar^s;  t' < j:  lam^< += (-dt Irow)^dag S^>,  lam^> += (dt Irow)^dag S^<
          // for this pass (column factors in registers), then for the earlier pass (from LDS,
          // read here in every row: the barrier keeps the compiler from holding them in
          // registers across the loop, which would leave room for one wavefront per SIMD only)
          auto update = [&](const cplx* SRr, const cplx* Irr, auto col_ib, auto col_sg, auto col_sl) {
            cplx A[NBB], X[NBB];
#pragma unroll
            for (int e = 0; e < NBB; ++e) A[e] = cscal(SRr[e], dt);
#pragma unroll
            for (int sc = 0; sc < 2; ++sc) {
#pragma unroll
              for (int e = 0; e < NBB; ++e) X[e] = col_ib(sc * NBB + e);
              mm_acc_adag<NB>(L + sc * NBB, A, X);
            }
            if (rv) {
#pragma unroll
              for (int e = 0; e < NBB; ++e) A[e] = cscal(Irr[e], -dt);
#pragma unroll
              for (int e = 0; e < NBB; ++e) X[e] = col_sg(e);
              mm_acc_adag<NB>(L, A, X);
#pragma unroll
              for (int e = 0; e < NBB; ++e) A[e] = cscal(Irr[e], dt);
#pragma unroll
              for (int e = 0; e < NBB; ++e) X[e] = col_sl(e);
              mm_acc_adag<NB>(L + NBB, A, X);
            }
          };
          update(SR, Irow, [&](int c) { return Ib[c]; }, [&](int e) { return Sg[e]; }, [&](int e) { return Sl[e]; });
          asm volatile("" ::: "memory");
          cplx SR1[NBB], Irow1[NBB];
#pragma unroll
          for (int e = 0; e < NBB; ++e) {
            SR1[e] = sk1[(2 * NBB + e) * d.Tp + j];
            Irow1[e] = cadd(Ibar1[rowbuf_idx(d, k, e, j)], Ibar1[rowbuf_idx(d, k, NBB + e, j)]);
          }
          update(SR1, Irow1, [&](int c) { return xI[c * 64 + lane]; }, [&](int e) { return xS[(NBB + e) * 64 + lane]; },
                 [&](int e) { return xS[e * 64 + lane]; });
          if (v) {
#pragma unroll
            for (int c = 0; c < C; ++c) store_stream(lk + off + 64 * c, L[c]);
          }
        }
        if (rv) {
          // Sigma adjoints of the row term (in lane)
          cplx x[NBB], y[NBB];
          mat_zero<NB>(x);
          mat_zero<NB>(y);
          mm_acc<NB>(x, Irow, G + NBB);  // Irow G^>  -> Sbar^<
          mm_acc<NB>(y, Irow, G);        // Irow G^<  -> -Sbar^>
#pragma unroll
          for (int e = 0; e < NBB; ++e) {
            acc[e] = cadd(acc[e], cscal(x[e], dt));
            acc[NBB + e] = csub(acc[NBB + e], cscal(y[e], dt));
          }
        }
        // SRbar_j partial: sum_s Ibar^s G^s^dag (zero where no block is stored)
        cplx q[NBB];
        mat_zero<NB>(q);
        mm_acc_bdag<NB>(q, Ib, G);
        mm_acc_bdag<NB>(q, Ib + NBB, G + NBB);
        if constexpr (NBB == 4) {
          // the four components are the four groups of one reduce-scatter
          double xg[4][2];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            xg[e][0] = q[e].x * dt;
            xg[e][1] = q[e].y * dt;
          }
          reduce_rows<4>(xg);
          const int e = reduced_row<4>(lane);
          if (e >= 0) st[e * ROWS_ST + (j - cb)] = cmk(xg[0][0], xg[0][1]);
        } else {
          double rt[1][2 * NBB];
#pragma unroll
          for (int e = 0; e < NBB; ++e) {
            rt[0][2 * e] = q[e].x * dt;
            rt[0][2 * e + 1] = q[e].y * dt;
          }
          reduce_rows<1>(rt);
          if (reduced_row<1>(lane) >= 0) {
#pragma unroll
            for (int e = 0; e < NBB; ++e) st[e * ROWS_ST + (j - cb)] = cmk(rt[0][2 * e], rt[0][2 * e + 1]);
          }
        }
      };
      if (j >= 64 * s + 64)
        row(BoolTag<false>{});
      else
        row(BoolTag<true>{});
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
        if (colv) sbar_col[rowbuf_idx(d, k, c0 + c, tp)] = a;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ end points and equal time
// One block per k. Forward terms (times dt) of output t' < m:
//   +1/2 SR_m R_{t'} - 1/2 SR_0 G0(t') + [t'>0](-1/2 S^s_{t'} GR_{t't'} + 1/2 S^s_0 GR0(t')),
//   G0(0) = G_00, G0(t') = -G_{t'0}^dag, GR = G^> - G^<;
// and the equal-time output (both components the same matrix)
//   I_d = dt sum_j a_j [S^>_j Gjm^< - S^<_j Gjm^>],  Gjm = -R_j^dag (j < m), R_m (j = m).
// Produces the complete Sigma adjoint row sbar (lesser, greater), the adjoint of the current
// row Rbar (overwritten), and the end-point updates of the adjoint history.
template <int NB>
__global__ __launch_bounds__(256) void k_adj_row(Dims d, const cplx* __restrict__ row64, const cplx* __restrict__ sig,
                                                 const cplx* __restrict__ col0, const cplx* __restrict__ diag,
                                                 const cplx* __restrict__ Ibar, const cplx* __restrict__ Dbar,
                                                 const cplx* __restrict__ sbar_col,
                                                 const cplx* __restrict__ sbar_rowpart, cplx* __restrict__ sbar,
                                                 cplx* __restrict__ Rbar, cplx* __restrict__ lam, int m, double dt) {
  constexpr int NBB = NB * NB, C = 2 * NBB;
  constexpr int NR = 4 * NBB;  // reductions: SRbar_m, SRbar_0, Sbar^<_0, Sbar^>_0
  __shared__ cplx wred[4][NR];
  __shared__ cplx tot[NR];
  int k = blockIdx.x;
  auto S = [&](int sc, int e, int j) { return sig[sig_idx(d, k, sc, e, j)]; };
  cplx SRm[NBB], SR0[NBB], Sl0[NBB], Sg0[NBB], Id[NBB];
#pragma unroll
  for (int e = 0; e < NBB; ++e) {
    SRm[e] = S(2, e, m);
    SR0[e] = S(2, e, 0);
    Sl0[e] = S(0, e, 0);
    Sg0[e] = S(1, e, 0);
  }
  // adjoint of the equal-time matrix: Ibar^<(m) + Ibar^>(m) + Dbar + Dbar^dag
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      int e = a * NB + b;
      cplx v = cadd(Ibar[rowbuf_idx(d, k, e, m)], Ibar[rowbuf_idx(d, k, NBB + e, m)]);
      v = cadd(v, Dbar[(int64_t)k * NBB + e]);
      v = cadd(v, cconj(Dbar[(int64_t)k * NBB + b * NB + a]));
      Id[e] = v;
    }
  // phase 1: reductions over t' of the j = 0 and j = m Sigma adjoints
  cplx r[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) r[i] = czero();
  for (int tp = threadIdx.x; tp < m; tp += blockDim.x) {
    cplx Ib[C], Rr[C], G0[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      Ib[c] = Ibar[rowbuf_idx(d, k, c, tp)];
      Rr[c] = row64[row64_idx(d, m, k, c, tp)];
    }
    if (tp == 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) G0[c] = col0[rowbuf_idx(d, k, c, 0)];
    } else {
#pragma unroll
      for (int sc = 0; sc < 2; ++sc)
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b)
            G0[sc * NBB + a * NB + b] = cneg(cconj(col0[rowbuf_idx(d, k, sc * NBB + b * NB + a, tp)]));
    }
    cplx t[NBB];
#pragma unroll
    for (int sc = 0; sc < 2; ++sc) {
      // SRbar_m += 1/2 dt Ibar^s R^s^dag ;  SRbar_0 -= 1/2 dt Ibar^s G0^s^dag
      mat_zero<NB>(t);
      mm_acc_bdag<NB>(t, Ib + sc * NBB, Rr + sc * NBB);
#pragma unroll
      for (int e = 0; e < NBB; ++e) r[e] = cadd(r[e], cscal(t[e], 0.5 * dt));
      mat_zero<NB>(t);
      mm_acc_bdag<NB>(t, Ib + sc * NBB, G0 + sc * NBB);
#pragma unroll
      for (int e = 0; e < NBB; ++e) r[NBB + e] = csub(r[NBB + e], cscal(t[e], 0.5 * dt));
    }
    if (tp > 0) {
      // Sbar^s_0 += 1/2 dt Ibar^s GR0^dag
      cplx GR0[NBB];
#pragma unroll
      for (int e = 0; e < NBB; ++e) GR0[e] = csub(G0[NBB + e], G0[e]);
#pragma unroll
      for (int sc = 0; sc < 2; ++sc) {
        mat_zero<NB>(t);
        mm_acc_bdag<NB>(t, Ib + sc * NBB, GR0);
#pragma unroll
        for (int e = 0; e < NBB; ++e) r[(2 + sc) * NBB + e] = cadd(r[(2 + sc) * NBB + e], cscal(t[e], 0.5 * dt));
      }
    }
  }
  {
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      cplx v = cmk(wave_sum(r[i].x), wave_sum(r[i].y));
      if (lane == 0) wred[wv][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < NR) {
      int i = threadIdx.x;
      tot[i] = cadd(cadd(wred[0][i], wred[1][i]), cadd(wred[2][i], wred[3][i]));
    }
    __syncthreads();
  }
  // phase 2: every t' = j in 0..m
  for (int tp = threadIdx.x; tp <= m; tp += blockDim.x) {
    cplx sb[C], srb[NBB], rb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) rb[c] = czero();
#pragma unroll
    for (int e = 0; e < NBB; ++e) srb[e] = czero();
    if (tp < m) {
#pragma unroll
      for (int c = 0; c < C; ++c) sb[c] = sbar_col[rowbuf_idx(d, k, c, tp)];
      int ns = (tp >> 6) + 1;
      for (int s = 0; s < ns; ++s) {
        const cplx* rp = sbar_rowpart + ((int64_t)k * d.Smax + s) * NBB * d.Tp;
#pragma unroll
        for (int e = 0; e < NBB; ++e) srb[e] = cadd(srb[e], rp[(int64_t)e * d.Tp + tp]);
      }
    } else {
#pragma unroll
      for (int c = 0; c < C; ++c) sb[c] = czero();
    }
    if (tp < m) {
      cplx Ib[C], G0[C], Gbar0[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        Ib[c] = Ibar[rowbuf_idx(d, k, c, tp)];
        Gbar0[c] = czero();
      }
      if (tp == 0) {
#pragma unroll
        for (int c = 0; c < C; ++c) G0[c] = col0[rowbuf_idx(d, k, c, 0)];
      } else {
#pragma unroll
        for (int sc = 0; sc < 2; ++sc)
#pragma unroll
          for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
              G0[sc * NBB + a * NB + b] = cneg(cconj(col0[rowbuf_idx(d, k, sc * NBB + b * NB + a, tp)]));
      }
#pragma unroll
      for (int sc = 0; sc < 2; ++sc) {
        // Rbar^s_{t'} += 1/2 dt SR_m^dag Ibar^s ;  G0bar^s -= 1/2 dt SR_0^dag Ibar^s
        cplx t[NBB];
        mat_zero<NB>(t);
        mm_acc_adag<NB>(t, SRm, Ib + sc * NBB);
#pragma unroll
        for (int e = 0; e < NBB; ++e) rb[sc * NBB + e] = cadd(rb[sc * NBB + e], cscal(t[e], 0.5 * dt));
        mat_zero<NB>(t);
        mm_acc_adag<NB>(t, SR0, Ib + sc * NBB);
#pragma unroll
        for (int e = 0; e < NBB; ++e) Gbar0[sc * NBB + e] = csub(Gbar0[sc * NBB + e], cscal(t[e], 0.5 * dt));
      }
      if (tp > 0) {
        cplx GRtt[NBB], GRbar[NBB], GR0bar[NBB];
#pragma unroll
        for (int e = 0; e < NBB; ++e) {
          GRtt[e] = csub(diag[rowbuf_idx(d, k, NBB + e, tp)], diag[rowbuf_idx(d, k, e, tp)]);
          GRbar[e] = czero();
          GR0bar[e] = czero();
        }
#pragma unroll
        for (int sc = 0; sc < 2; ++sc) {
          cplx St[NBB], S0[NBB], t[NBB];
#pragma unroll
          for (int e = 0; e < NBB; ++e) {
            St[e] = S(sc, e, tp);
            S0[e] = sc ? Sg0[e] : Sl0[e];
          }
          // -1/2 S^s_{t'} GR_{t't'}:  Sbar^s_{t'} -= 1/2 dt Ibar^s GRtt^dag,  GRbar -= 1/2 dt S^s_{t'}^dag Ibar^s
          mat_zero<NB>(t);
          mm_acc_bdag<NB>(t, Ib + sc * NBB, GRtt);
#pragma unroll
          for (int e = 0; e < NBB; ++e) sb[sc * NBB + e] = csub(sb[sc * NBB + e], cscal(t[e], 0.5 * dt));
          mat_zero<NB>(t);
          mm_acc_adag<NB>(t, St, Ib + sc * NBB);
#pragma unroll
          for (int e = 0; e < NBB; ++e) GRbar[e] = csub(GRbar[e], cscal(t[e], 0.5 * dt));
          // +1/2 S^s_0 GR0:  GR0bar += 1/2 dt S^s_0^dag Ibar^s
          mat_zero<NB>(t);
          mm_acc_adag<NB>(t, S0, Ib + sc * NBB);
#pragma unroll
          for (int e = 0; e < NBB; ++e) GR0bar[e] = cadd(GR0bar[e], cscal(t[e], 0.5 * dt));
        }
#pragma unroll
        for (int e = 0; e < NBB; ++e) {
          Gbar0[NBB + e] = cadd(Gbar0[NBB + e], GR0bar[e]);
          Gbar0[e] = csub(Gbar0[e], GR0bar[e]);
        }
        // GR_{t't'} = G^>_{t't'} - G^<_{t't'}: adjoint history diagonal block
#pragma unroll
        for (int e = 0; e < NBB; ++e) {
          int64_t il = hist_idx(d, k, e, tp, tp), ig = hist_idx(d, k, NBB + e, tp, tp);
          lam[il] = csub(lam[il], GRbar[e]);
          lam[ig] = cadd(lam[ig], GRbar[e]);
        }
        // G0 = -G_{t'0}^dag
#pragma unroll
        for (int sc = 0; sc < 2; ++sc)
#pragma unroll
          for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              int64_t i0 = hist_idx(d, k, sc * NBB + a * NB + b, tp, 0);
              lam[i0] = csub(lam[i0], cconj(Gbar0[sc * NBB + b * NB + a]));
            }
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) {
          int64_t i0 = hist_idx(d, k, c, 0, 0);
          lam[i0] = cadd(lam[i0], Gbar0[c]);
        }
      }
    }
    // equal-time term, node j = tp
    {
      int j = tp;
      double wgt = (m == 0) ? 0.0 : ((j == 0 || j == m) ? 0.5 : 1.0);
      cplx Rl[NBB], Rg[NBB], Gl[NBB], Gg[NBB];
#pragma unroll
      for (int e = 0; e < NBB; ++e) {
        Rl[e] = row64[row64_idx(d, m, k, e, j)];
        Rg[e] = row64[row64_idx(d, m, k, NBB + e, j)];
      }
      if (j < m) {
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            Gl[a * NB + b] = cneg(cconj(Rl[b * NB + a]));
            Gg[a * NB + b] = cneg(cconj(Rg[b * NB + a]));
          }
      } else {
#pragma unroll
        for (int e = 0; e < NBB; ++e) {
          Gl[e] = Rl[e];
          Gg[e] = Rg[e];
        }
      }
      double f = dt * wgt;
      cplx t[NBB], Glb[NBB], Ggb[NBB];
      // Sbar^>_j += f Id Gl^dag ;  Sbar^<_j -= f Id Gg^dag
      mat_zero<NB>(t);
      mm_acc_bdag<NB>(t, Id, Gl);
#pragma unroll
      for (int e = 0; e < NBB; ++e) sb[NBB + e] = cadd(sb[NBB + e], cscal(t[e], f));
      mat_zero<NB>(t);
      mm_acc_bdag<NB>(t, Id, Gg);
#pragma unroll
      for (int e = 0; e < NBB; ++e) sb[e] = csub(sb[e], cscal(t[e], f));
      // Glbar = f S^>_j^dag Id ;  Ggbar = -f S^<_j^dag Id
      cplx Sj[NBB];
#pragma unroll
      for (int e = 0; e < NBB; ++e) Sj[e] = S(1, e, j);
      mat_zero<NB>(Glb);
      mm_acc_adag<NB>(Glb, Sj, Id);
#pragma unroll
      for (int e = 0; e < NBB; ++e) Sj[e] = S(0, e, j);
      mat_zero<NB>(Ggb);
      mm_acc_adag<NB>(Ggb, Sj, Id);
#pragma unroll
      for (int e = 0; e < NBB; ++e) {
        Glb[e] = cscal(Glb[e], f);
        Ggb[e] = cscal(Ggb[e], -f);
      }
      if (j < m) {
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            rb[a * NB + b] = csub(rb[a * NB + b], cconj(Glb[b * NB + a]));
            rb[NBB + a * NB + b] = csub(rb[NBB + a * NB + b], cconj(Ggb[b * NB + a]));
          }
      } else {
#pragma unroll
        for (int e = 0; e < NBB; ++e) {
          rb[e] = cadd(rb[e], Glb[e]);
          rb[NBB + e] = cadd(rb[NBB + e], Ggb[e]);
        }
      }
    }
    if (tp == 0) {
#pragma unroll
      for (int e = 0; e < NBB; ++e) {
        srb[e] = cadd(srb[e], tot[NBB + e]);
        sb[e] = cadd(sb[e], tot[2 * NBB + e]);
        sb[NBB + e] = cadd(sb[NBB + e], tot[3 * NBB + e]);
      }
    }
    if (tp == m) {
#pragma unroll
      for (int e = 0; e < NBB; ++e) srb[e] = cadd(srb[e], tot[e]);
    }
    // Sigma^R = Sigma^> - Sigma^<
#pragma unroll
    for (int e = 0; e < NBB; ++e) {
      sbar[(((int64_t)k * 2 + 0) * NBB + e) * d.Tp + tp] = csub(sb[e], srb[e]);
      sbar[(((int64_t)k * 2 + 1) * NBB + e) * d.Tp + tp] = cadd(sb[NBB + e], srb[e]);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) Rbar[rowbuf_idx(d, k, c, tp)] = rb[c];
  }
}

// ------------------------------------------------------------------ self-energy adjoint
// Forward per (t_j, ab): g = N_k^{-1} F^+ G,  s^< = c g^<^2 conj(g^>),  s^> = c g^>^2 conj(g^<),
// Sigma = F^- s, with c = -U^2 and F^{+-} the index transforms with e^{+-2 pi i j.R/n}.
// Adjoint: sbar(R) = F^+ Sigmabar (no 1/N_k),
//   gbar^< = 2 c conj(g^<) g^> sbar^< + c g^>^2 conj(sbar^>),
//   gbar^> = c g^<^2 conj(sbar^<) + 2 c conj(g^>) g^< sbar^>,
//   Gbar(k) += N_k^{-1} F^- gbar,   dL/dU += sum Re conj(sbar) ds/dU,  ds/dU = 2 s / U.
template <int NB>
__global__ __launch_bounds__(256) void k_adj_sigma(Dims d, const cplx* __restrict__ row64,
                                                   const cplx* __restrict__ sbar, cplx* __restrict__ Rbar,
                                                   double* __restrict__ ubar_part, int m, double U, int corr) {
  constexpr int NBB = NB * NB;
  constexpr int PT = 4;  // k points per thread (N_k <= 1024)
  extern __shared__ cplx lds[];
  __shared__ double ured[256];
  __shared__ cplx twx[64], twy[64];
  cplx* xl = lds;
  cplx* xg = lds + d.nk;
  cplx* tl = lds + 2 * d.nk;
  cplx* tg = lds + 3 * d.nk;
  int total = (m + 1) * NBB;
  int per = (total + 7) >> 3;
  int item = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  double up = 0.0;
  if (item < total) {
    int j = item / NBB, ab = item - (item / NBB) * NBB;
    int t = threadIdx.x;
    int nx = d.nkx, ny = d.nky, nk = d.nk;
    fill_roots(twx, nx);
    fill_roots(twy, ny);
    for (int k = t; k < nk; k += 256) {
      xl[k] = row64[row64_idx(d, m, k, ab, j)];
      xg[k] = row64[row64_idx(d, m, k, NBB + ab, j)];
    }
    __syncthreads();
    grid_dft(xl, xg, tl, tg, nx, ny, twx, twy, +1, 1.0 / nk);  // g(R)
    cplx ra[PT], rb[PT];
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      int o = t + 256 * i;
      ra[i] = o < nk ? xl[o] : czero();
      rb[i] = o < nk ? xg[o] : czero();
    }
    __syncthreads();
    for (int k = t; k < nk; k += 256) {
      xl[k] = sbar[(((int64_t)k * 2 + 0) * NBB + ab) * d.Tp + j];
      xg[k] = sbar[(((int64_t)k * 2 + 1) * NBB + ab) * d.Tp + j];
    }
    __syncthreads();
    grid_dft(xl, xg, tl, tg, nx, ny, twx, twy, +1, 1.0);  // sbar(R)
    double cc = -U * U;
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      int o = t + 256 * i;
      if (o >= nk) continue;
      cplx a = ra[i], b = rb[i], sl = xl[o], sg = xg[o];
      cplx ga = czero(), gb = czero();
      if (corr) {
        // gbar^< = 2c conj(a) b sl + c b^2 conj(sg);  gbar^> = c a^2 conj(sl) + 2c conj(b) a sg
        ga = cadd(cscal(cmul(cmul(cconj(a), b), sl), 2.0 * cc), cscal(cmul(cmul(b, b), cconj(sg)), cc));
        gb = cadd(cscal(cmul(cmul(a, a), cconj(sl)), cc), cscal(cmul(cmul(cconj(b), a), sg), 2.0 * cc));
        // ds^</dU = -2U a^2 conj(b), ds^>/dU = -2U b^2 conj(a)
        cplx dsl = cscal(cmul(cmul(a, a), cconj(b)), -2.0 * U);
        cplx dsg = cscal(cmul(cmul(b, b), cconj(a)), -2.0 * U);
        up += sl.x * dsl.x + sl.y * dsl.y + sg.x * dsg.x + sg.y * dsg.y;
      }
      xl[o] = ga;
      xg[o] = gb;
    }
    __syncthreads();
    grid_dft(xl, xg, tl, tg, nx, ny, twx, twy, -1, 1.0 / nk);
    for (int k = t; k < nk; k += 256) {
      int64_t il = rowbuf_idx(d, k, ab, j), ig = rowbuf_idx(d, k, NBB + ab, j);
      Rbar[il] = cadd(Rbar[il], xl[k]);
      Rbar[ig] = cadd(Rbar[ig], xg[k]);
    }
  }
  ured[threadIdx.x] = up;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) ured[threadIdx.x] += ured[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) ubar_part[blockIdx.x] = ured[0];
}

// ------------------------------------------------------------------ update adjoint
// Forward (t' < m):  G_m(t') = V G_{m-1}(t') + Phi Ibar(t'),  Ibar = f1 I_{m-1} + f2 I_c;
// t' = m:  G_m(m) = (i rho_m, -i (1 - rho_m)),  rho_m = V rho_{m-1} V^dag - dt W Dbar W^dag,
// Dbar = g1 D_{m-1} + g2 D_c. One block per k.
template <int NB>
__global__ __launch_bounds__(256) void k_adj_update(Dims d, const cplx* __restrict__ lam_rowm,
                                                    const cplx* __restrict__ Gbar_row, cplx* __restrict__ lam,
                                                    const cplx* __restrict__ row64, const cplx* __restrict__ props,
                                                    const cplx* __restrict__ Iprev, const cplx* __restrict__ Ic,
                                                    const cplx* __restrict__ rho_prev, const cplx* __restrict__ Dprev,
                                                    const cplx* __restrict__ Dc, cplx* __restrict__ Ibar_prev,
                                                    cplx* __restrict__ Ibar_c, cplx* __restrict__ rhobar,
                                                    cplx* __restrict__ rhobar_prev, cplx* __restrict__ Dbar_prev,
                                                    cplx* __restrict__ Dbar_c, cplx* __restrict__ pbar, int m,
                                                    double dt, int corrector) {
  constexpr int NBB = NB * NB, C = 2 * NBB;
  __shared__ cplx lds[2 * NBB * 256];
  int k = blockIdx.x;
  const cplx* P = props + (int64_t)k * 3 * NBB;
  cplx V[NBB], W[NBB], Phi[NBB];
#pragma unroll
  for (int e = 0; e < NBB; ++e) {
    V[e] = P[e];
    W[e] = P[NBB + e];
    Phi[e] = P[2 * NBB + e];
  }
  double f1 = corrector ? 0.5 : 1.0;
  cplx Vb[NBB], Pb[NBB];  // per-thread partial V-bar, Phi-bar
#pragma unroll
  for (int e = 0; e < NBB; ++e) {
    Vb[e] = czero();
    Pb[e] = czero();
  }
  auto gbar = [&](int c, int tp) {
    cplx g = Gbar_row ? Gbar_row[rowbuf_idx(d, k, c, tp)] : czero();
    if (lam_rowm) g = cadd(g, lam_rowm[hist_idx(d, k, c, m, tp)]);
    return g;
  };
  for (int tp = threadIdx.x; tp < m; tp += blockDim.x) {
    cplx Gb[C], Go[C], Ib[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      Gb[c] = gbar(c, tp);
      Go[c] = row64[row64_idx(d, m - 1, k, c, tp)];
      cplx ip = Iprev[rowbuf_idx(d, k, c, tp)];
      Ib[c] = corrector ? cscal(cadd(ip, Ic[rowbuf_idx(d, k, c, tp)]), 0.5) : ip;
    }
#pragma unroll
    for (int sc = 0; sc < 2; ++sc) {
      cplx t[NBB], u[NBB];
      // lam_{m-1}(t') += V^dag Gbar
      mat_zero<NB>(t);
      mm_acc_adag<NB>(t, V, Gb + sc * NBB);
#pragma unroll
      for (int e = 0; e < NBB; ++e) {
        int64_t i = hist_idx(d, k, sc * NBB + e, m - 1, tp);
        lam[i] = cadd(lam[i], t[e]);
      }
      // Ibar_{m-1} += f1 Phi^dag Gbar ;  Ibar_c = 1/2 Phi^dag Gbar
      mat_zero<NB>(u);
      mm_acc_adag<NB>(u, Phi, Gb + sc * NBB);
#pragma unroll
      for (int e = 0; e < NBB; ++e) {
        int64_t i = rowbuf_idx(d, k, sc * NBB + e, tp);
        Ibar_prev[i] = cadd(Ibar_prev[i], cscal(u[e], f1));
        if (corrector) Ibar_c[i] = cscal(u[e], 0.5);
      }
      // Vbar += Gbar Go^dag ;  Phibar += Gbar Ib^dag
      mm_acc_bdag<NB>(Vb, Gb + sc * NBB, Go + sc * NBB);
      mm_acc_bdag<NB>(Pb, Gb + sc * NBB, Ib + sc * NBB);
    }
  }
  if (corrector && threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < C; ++c) Ibar_c[rowbuf_idx(d, k, c, m)] = czero();  // I_c(t_m, t_m) only enters D_c
  // reduce V-bar, Phi-bar over the block
  {
    int t = threadIdx.x;
#pragma unroll
    for (int e = 0; e < NBB; ++e) {
      lds[e * 256 + t] = Vb[e];
      lds[(NBB + e) * 256 + t] = Pb[e];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s)
#pragma unroll
        for (int i = 0; i < 2 * NBB; ++i) lds[i * 256 + t] = cadd(lds[i * 256 + t], lds[i * 256 + t + s]);
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int e = 0; e < NBB; ++e) {
      Vb[e] = lds[e * 256];
      Pb[e] = lds[(NBB + e) * 256];
    }
    // equal-time block: G^< = i rho, G^> = -i + i rho  ->  rhobar += -i (Gbar^<_mm + Gbar^>_mm)
    cplx rb[NBB], r0[NBB], Db[NBB], Wb[NBB], t1[NBB], t2[NBB];
#pragma unroll
    for (int e = 0; e < NBB; ++e) {
      cplx g = cadd(gbar(e, m), gbar(NBB + e, m));
      rb[e] = cadd(rhobar[(int64_t)k * NBB + e], cmk(g.y, -g.x));
      rhobar[(int64_t)k * NBB + e] = rb[e];
      r0[e] = rho_prev[(int64_t)k * NBB + e];
      cplx dp = Dprev[(int64_t)k * NBB + e];
      Db[e] = corrector ? cscal(cadd(dp, Dc[(int64_t)k * NBB + e]), 0.5) : dp;
      Wb[e] = czero();
    }
    // rho = V r0 V^dag:  r0bar += V^dag rb V ;  Vbar += rb V r0^dag + rb^dag V r0
    mat_zero<NB>(t1);
    mm_acc_adag<NB>(t1, V, rb);
    mat_zero<NB>(t2);
    mm_acc<NB>(t2, t1, V);
#pragma unroll
    for (int e = 0; e < NBB; ++e) rhobar_prev[(int64_t)k * NBB + e] = cadd(rhobar_prev[(int64_t)k * NBB + e], t2[e]);
    mat_zero<NB>(t1);
    mm_acc<NB>(t1, rb, V);
    mm_acc_bdag<NB>(Vb, t1, r0);
    cplx rbd[NBB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) rbd[a * NB + b] = cconj(rb[b * NB + a]);
    mat_zero<NB>(t1);
    mm_acc<NB>(t1, rbd, V);
    mm_acc<NB>(Vb, t1, r0);
    // -dt W Db W^dag:  Wbar += -dt (rb W Db^dag + rb^dag W Db) ;  Dbbar = -dt W^dag rb W
    mat_zero<NB>(t1);
    mm_acc<NB>(t1, rb, W);
    mat_zero<NB>(t2);
    mm_acc_bdag<NB>(t2, t1, Db);
    mat_zero<NB>(t1);
    mm_acc<NB>(t1, rbd, W);
    mm_acc<NB>(t2, t1, Db);
#pragma unroll
    for (int e = 0; e < NBB; ++e) Wb[e] = cscal(t2[e], -dt);
    mat_zero<NB>(t1);
    mm_acc_adag<NB>(t1, W, rb);
    mat_zero<NB>(t2);
    mm_acc<NB>(t2, t1, W);
#pragma unroll
    for (int e = 0; e < NBB; ++e) {
      cplx x = cscal(t2[e], -dt);
      if (corrector) {
        Dbar_prev[(int64_t)k * NBB + e] = cadd(Dbar_prev[(int64_t)k * NBB + e], cscal(x, 0.5));
        Dbar_c[(int64_t)k * NBB + e] = cscal(x, 0.5);
      } else {
        Dbar_prev[(int64_t)k * NBB + e] = cadd(Dbar_prev[(int64_t)k * NBB + e], x);
      }
    }
    cplx* pb = pbar + (int64_t)k * 3 * NBB;
#pragma unroll
    for (int e = 0; e < NBB; ++e) {
      pb[e] = Vb[e];
      pb[NBB + e] = Wb[e];
      pb[2 * NBB + e] = Pb[e];
    }
  }
}

// ------------------------------------------------------------------ propagator adjoint
// M = [[-i hbar dt, dt 1], [0, 0]];  V = exp(M)_tl,  Phi = -i exp(M)_tr,  Vh = exp(M/2)_tl.
// For E = exp(X) the adjoint is Xbar = L(X^dag, Ebar), the Frechet derivative of exp at X^dag
// in the direction Ebar, read off the top-right block of exp([[X^dag, Ebar], [0, X^dag]]).
// Ebar = [[Vbar, i Phibar], [0, 0]] for exp(M), [[Vhbar, 0], [0, 0]] for exp(M/2);
// hbarbar = i dt (Mbar)_tl. One wavefront per k (block matrices up to 8 x 8: nb <= 2).
template <int NB>
__global__ __launch_bounds__(256) void k_adj_props(Dims d, const cplx* __restrict__ hop, const cplx* __restrict__ hf,
                                                   const cplx* __restrict__ pbar, double Ax, double Ay, double polx,
                                                   double poly, double dt, double* __restrict__ kpart) {
  constexpr int NBB = NB * NB, N2 = 2 * NB, B2 = 2 * N2, BB = B2 * B2;
  static_assert(BB <= 64, "adjoint propagators support nb <= 2");
  __shared__ cplx sX[4][BB], sE[4][BB];
  __shared__ cplx hb[4][NBB];
  int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int k = blockIdx.x * 4 + wv;
  bool kval = k < d.nk;
  int r = lane / B2, c = lane - (lane / B2) * B2;
  bool act = kval && lane < BB;
  cplx h[NBB];
  if (kval) {
    bloch_h0<NB>(hop, d.nkx, d.nky, k, Ax, Ay, h);
#pragma unroll
    for (int e = 0; e < NBB; ++e) h[e] = cadd(h[e], hf[e]);
  }
  const cplx* pb = pbar + (int64_t)(kval ? k : 0) * 3 * NBB;
  // M (N2 x N2) element (i, j)
  auto Mel = [&](int i, int j, double sc) -> cplx {
    if (i < NB && j < NB) return cscal(cmuli(h[i * NB + j]), -dt * sc);
    if (i < NB && j == i + NB) return cmk(dt * sc, 0.0);
    return czero();
  };
  cplx mbar = czero();  // (Mbar)_tl element of lane (r, c) when r, c < NB
  for (int pass = 0; pass < 2; ++pass) {
    double sc = pass == 0 ? 1.0 : 0.5;
    // Ebar (N2 x N2)
    auto Ebar = [&](int i, int j) -> cplx {
      if (pass == 0) {
        if (i < NB && j < NB) return pb[i * NB + j];
        if (i < NB && j >= NB) return cmuli(pb[2 * NBB + i * NB + (j - NB)]);
        return czero();
      }
      if (i < NB && j < NB) return pb[NBB + i * NB + j];
      return czero();
    };
    // block matrix B = [[M^dag, Ebar/nE], [0, M^dag]] with the direction normalised
    double ne = 0.0;
    if (act && r < N2 && c >= N2) ne = cabs2(Ebar(r, c - N2));
    ne = sqrt(wave_sum(ne));
    double inv_ne = ne > 0.0 ? 1.0 / ne : 0.0;
    cplx x = czero();
    if (act) {
      if (r < N2 && c < N2) x = cconj(Mel(c, r, sc));
      else if (r >= N2 && c >= N2) x = cconj(Mel(c - N2, r - N2, sc));
      else if (r < N2 && c >= N2) x = cscal(Ebar(r, c - N2), inv_ne);
    }
    double nrm = sqrt(wave_sum(act ? cabs2(x) : 0.0));
    int s = 0;
    while (nrm > ldexp(0.25, s) && s < 60) ++s;
    x = cscal(x, ldexp(1.0, -s));
    cplx id = cmk((act && r == c) ? 1.0 : 0.0, 0.0);
    if (lane < BB) sX[wv][lane] = x;
    cplx e = id;
    if (lane < BB) sE[wv][lane] = e;
    wave_sync();  // every LDS array here is per wavefront
    for (int n = 18; n >= 1; --n) {
      cplx acc = czero();
      if (lane < BB)
#pragma unroll
        for (int l = 0; l < B2; ++l) cmac(acc, sX[wv][r * B2 + l], sE[wv][l * B2 + c]);
      wave_sync();  // every LDS array here is per wavefront
      e = cadd(id, cscal(acc, 1.0 / n));
      if (lane < BB) sE[wv][lane] = e;
      wave_sync();  // every LDS array here is per wavefront
    }
    for (int q = 0; q < s; ++q) {
      cplx acc = czero();
      if (lane < BB)
#pragma unroll
        for (int l = 0; l < B2; ++l) cmac(acc, sE[wv][r * B2 + l], sE[wv][l * B2 + c]);
      wave_sync();  // every LDS array here is per wavefront
      e = acc;
      if (lane < BB) sE[wv][lane] = e;
      wave_sync();  // every LDS array here is per wavefront
    }
    // top-right block, top-left (NB x NB) sub-block of L: (r, c - N2) with r, c - N2 < NB
    if (act && r < NB && c >= N2 && c - N2 < NB) mbar = cadd(mbar, cscal(e, ne * sc));
  }
  // hbarbar = i dt Mbar_tl
  if (act && r < NB && c >= N2 && c - N2 < NB) hb[wv][r * NB + (c - N2)] = cscal(cmuli(mbar), dt);
  wave_sync();  // every LDS array here is per wavefront
  if (kval && lane == 0) {
    // dL/dhf_aa += Re hbarbar_aa ;  dL/dA += Re sum conj(hbarbar) dh0/dA, dh0/dA = -(pol . v)
    cplx vx[NBB], vy[NBB];
    bloch_vel<NB>(hop, d.nkx, d.nky, k, Ax, Ay, 0, vx);
    bloch_vel<NB>(hop, d.nkx, d.nky, k, Ax, Ay, 1, vy);
    double dA = 0.0;
#pragma unroll
    for (int e = 0; e < NBB; ++e) {
      cplx dh = cneg(cadd(cscal(vx[e], polx), cscal(vy[e], poly)));
      dA += hb[wv][e].x * dh.x + hb[wv][e].y * dh.y;
    }
#pragma unroll
    for (int a = 0; a < NB; ++a) kpart[(int64_t)k * (NB + 1) + a] = hb[wv][a * NB + a].x;
    kpart[(int64_t)k * (NB + 1) + NB] = dA;
  }
}

// ------------------------------------------------------------------ mean field and pulse
// hf_aa = U Re rho_loc,aa, rho_loc = N_k^{-1} sum_k [(1 - wb) rhoA(k) + wb rhoB(k)] (Hubbard);
// A(t_{m-1/2}) enters h0. One block: reduces the per-k partials, then scatters.
template <int NB>
__global__ __launch_bounds__(256) void k_adj_hf(Dims d, const double* __restrict__ kpart,
                                                const cplx* __restrict__ rhoA, const cplx* __restrict__ rhoB,
                                                double wb, int hf, double U, cplx* __restrict__ rbarA,
                                                cplx* __restrict__ rbarB, double dAdamp, double dAdomega,
                                                double* __restrict__ theta_bar) {
  __shared__ double red[(NB + 1 + NB) * 256];
  __shared__ double tot[NB + 1 + NB];
  int t = threadIdx.x;
  double p[NB + 1 + NB];
#pragma unroll
  for (int i = 0; i < 2 * NB + 1; ++i) p[i] = 0.0;
  for (int k = t; k < d.nk; k += 256) {
#pragma unroll
    for (int i = 0; i <= NB; ++i) p[i] += kpart[(int64_t)k * (NB + 1) + i];
#pragma unroll
    for (int a = 0; a < NB; ++a)
      p[NB + 1 + a] += (1.0 - wb) * rhoA[(int64_t)k * NB * NB + a * NB + a].x + wb * rhoB[(int64_t)k * NB * NB + a * NB + a].x;
  }
#pragma unroll
  for (int i = 0; i < 2 * NB + 1; ++i) red[i * 256 + t] = p[i];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s)
#pragma unroll
      for (int i = 0; i < 2 * NB + 1; ++i) red[i * 256 + t] += red[i * 256 + t + s];
    __syncthreads();
  }
  if (t < 2 * NB + 1) tot[t] = red[t * 256];
  __syncthreads();
  double inv = 1.0 / d.nk;
  if (hf) {
    for (int k = t; k < d.nk; k += 256)
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        double g = U * inv * tot[a];
        int64_t i = (int64_t)k * NB * NB + a * NB + a;
        if (1.0 - wb != 0.0) rbarA[i].x += (1.0 - wb) * g;
        if (wb != 0.0) rbarB[i].x += wb * g;
      }
  }
  if (t == 0) {
    double gU = 0.0;
    if (hf)
#pragma unroll
      for (int a = 0; a < NB; ++a) gU += tot[a] * tot[NB + 1 + a] * inv;
    theta_bar[0] += tot[NB] * dAdamp;
    theta_bar[1] += tot[NB] * dAdomega;
    theta_bar[2] += gU;
  }
}

__global__ __launch_bounds__(256) void k_adj_reduce_u(const double* __restrict__ part, int n,
                                                      double* __restrict__ theta_bar) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) theta_bar[2] += red[0];
}

// ------------------------------------------------------------------ observable seed
// O = N_k^{-1} sum_k Re tr[P_k rho_k], P_k the projector on band b of h0(k - A(T)) (or on
// orbital a). rhobar_T = P_k / N_k; for bands also dO/dA(T) by first-order perturbation
// theory, dP_b = sum_{c != b} (u_c u_c^dag dh u_b u_b^dag + h.c.) / (e_b - e_c), dh = -(pol.v) dA.
template <int NB>
__global__ __launch_bounds__(256) void k_adj_seed(Dims d, const cplx* __restrict__ hop, const cplx* __restrict__ rho,
                                                  double Ax, double Ay, double polx, double poly, int obs_id,
                                                  cplx* __restrict__ rhobar, double dAdamp, double dAdomega,
                                                  double* __restrict__ theta_bar) {
  constexpr int NBB = NB * NB;
  __shared__ double red[256];
  double inv = 1.0 / d.nk;
  double dOdA = 0.0;
  for (int k = threadIdx.x; k < d.nk; k += 256) {
    cplx Pm[NBB];
#pragma unroll
    for (int e = 0; e < NBB; ++e) Pm[e] = czero();
    if (obs_id >= KBE_DEV_OBS_NORB && obs_id < KBE_DEV_OBS_NORB + NB) {
      int a = obs_id - KBE_DEV_OBS_NORB;
      Pm[a * NB + a] = cmk(1.0, 0.0);
    } else {
      int b = obs_id - KBE_DEV_OBS_NBAND;
      cplx h[NBB], U[NBB], vx[NBB], vy[NBB], dh[NBB];
      double w[NB];
      bloch_h0<NB>(hop, d.nkx, d.nky, k, Ax, Ay, h);
      jacobi_eigh<NB>(h, w, U);
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) Pm[i * NB + j] = cmul(U[i * NB + b], cconj(U[j * NB + b]));
      bloch_vel<NB>(hop, d.nkx, d.nky, k, Ax, Ay, 0, vx);
      bloch_vel<NB>(hop, d.nkx, d.nky, k, Ax, Ay, 1, vy);
#pragma unroll
      for (int e = 0; e < NBB; ++e) dh[e] = cneg(cadd(cscal(vx[e], polx), cscal(vy[e], poly)));
      const cplx* r = rho + (int64_t)k * NBB;
      // Re tr(dP rho) = 2 Re sum_{c != b} <u_b|rho|u_c><u_c|dh|u_b> / (e_b - e_c)
      for (int c = 0; c < NB; ++c) {
        if (c == b) continue;
        cplx rbc = czero(), hcb = czero();
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            rbc = cadd(rbc, cmul(cmul(cconj(U[i * NB + b]), r[i * NB + j]), U[j * NB + c]));
            hcb = cadd(hcb, cmul(cmul(cconj(U[i * NB + c]), dh[i * NB + j]), U[j * NB + b]));
          }
        dOdA += 2.0 * cmul(rbc, hcb).x / (w[b] - w[c]);
      }
    }
#pragma unroll
    for (int e = 0; e < NBB; ++e) rhobar[(int64_t)k * NBB + e] = cscal(Pm[e], inv);
  }
  red[threadIdx.x] = dOdA * inv;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    theta_bar[0] += red[0] * dAdamp;
    theta_bar[1] += red[0] * dAdomega;
  }
}

// The row kernel stores the equal-time block as G^<(t_m, t_m) = i rho_m; multiplying by -i
// swaps the parts and flips one sign, so rho_m comes back bit for bit from the history.
template <int NB>
__global__ void k_adj_rho(Dims d, const void* __restrict__ hist, int m, cplx* __restrict__ rho) {
  constexpr int NBB = NB * NB;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.nk * NBB) return;
  int k = i / NBB, e = i - (i / NBB) * NBB;
  cplx g = static_cast<const cplx*>(hist)[hist_idx(d, k, e, m, m)];  // FP64 history
  rho[i] = cmk(g.y, -g.x);
}

// ------------------------------------------------------------------ launchers
template <int NB>
struct AdjLaunch {
  static hipError_t bulk(const Dims& d, const LaunchArgs& a, const AdjArgs& b, const cplx* Ibar, int m, int mode,
                         const cplx* sig1, const cplx* Ibar1, hipStream_t st) {
    if (m < 1) return hipSuccess;
    int ns = (m + 63) / 64;
    if (mode == ADJ_SUMS)
      hipLaunchKernelGGL((k_adj_bulk<NB, ADJ_SUMS>), dim3(ns * d.nk), dim3(256), 0, st, d, (const cplx*)a.hist,
                         b.lam, (const cplx*)a.sig, Ibar, (const cplx*)a.sig, Ibar, b.sbar_col, b.sbar_rowpart, m, a.dt);
    else
      hipLaunchKernelGGL((k_adj_bulk<NB, ADJ_FUSED>), dim3(ns * d.nk), dim3(256), 0, st, d, (const cplx*)a.hist,
                         b.lam, (const cplx*)a.sig, Ibar, sig1, Ibar1, b.sbar_col, b.sbar_rowpart, m, a.dt);
    return hipGetLastError();
  }
  static hipError_t row(const Dims& d, const LaunchArgs& a, const AdjArgs& b, const cplx* Ibar, const cplx* Dbar,
                        int m, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_row<NB>, dim3(d.nk), dim3(256), 0, st, d, (const cplx*)a.row64, (const cplx*)a.sig,
                       (const cplx*)a.col0, (const cplx*)a.diag, Ibar, Dbar, (const cplx*)b.sbar_col,
                       (const cplx*)b.sbar_rowpart, b.sbar, b.Rbar, b.lam, m, a.dt);
    return hipGetLastError();
  }
  static hipError_t sigma(const Dims& d, const LaunchArgs& a, const AdjArgs& b, int m, int* nblocks,
                          hipStream_t st) {
    int total = (m + 1) * NB * NB;
    int per = (total + 7) / 8;
    *nblocks = per * 8;
    size_t shm = (size_t)(4 * d.nk) * sizeof(cplx);
    hipLaunchKernelGGL(k_adj_sigma<NB>, dim3(per * 8), dim3(256), shm, st, d, (const cplx*)a.row64,
                       (const cplx*)b.sbar, b.Rbar, b.ubar_part, m, a.U, a.corr);
    return hipGetLastError();
  }
  static hipError_t update(const Dims& d, const LaunchArgs& a, const AdjArgs& b, int m, int corrector,
                           const cplx* Gbar_hist, const cplx* Gbar_row, const cplx* rho_prev, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_update<NB>, dim3(d.nk), dim3(256), 0, st, d, Gbar_hist, Gbar_row, b.lam,
                       (const cplx*)a.row64, (const cplx*)(corrector ? b.props_c : b.props_p),
                       (const cplx*)b.Ire_prev, (const cplx*)b.Ire_c, rho_prev, (const cplx*)a.D_prev,
                       (const cplx*)b.Dc, b.Ibar_prev, b.Ibar_c, corrector ? b.rhobar : b.rhobar_P,
                       b.rhobar_prev, b.Dbar_prev, b.Dbar_c, b.pbar, m, a.dt, corrector);
    return hipGetLastError();
  }
  static hipError_t props(const Dims& d, const LaunchArgs& a, const AdjArgs& b, const cplx* hf, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_props<NB>, dim3((d.nk + 3) / 4), dim3(256), 0, st, d, (const cplx*)a.hop, hf,
                       (const cplx*)b.pbar, a.Ax, a.Ay, a.polx, a.poly, a.dt, b.kpart);
    return hipGetLastError();
  }
  static hipError_t hf(const Dims& d, const LaunchArgs& a, const AdjArgs& b, const cplx* rA, const cplx* rB,
                       double wb, cplx* rbA, cplx* rbB, double dAdamp, double dAdomega, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_hf<NB>, dim3(1), dim3(256), 0, st, d, (const double*)b.kpart, rA, rB, wb, a.hf, a.U,
                       rbA, rbB, dAdamp, dAdomega, b.theta_bar);
    return hipGetLastError();
  }
  static hipError_t rho(const Dims& d, const void* hist, int m, cplx* out, hipStream_t st) {
    int n = d.nk * NB * NB;
    hipLaunchKernelGGL(k_adj_rho<NB>, dim3((n + 255) / 256), dim3(256), 0, st, d, hist, m, out);
    return hipGetLastError();
  }
  static hipError_t seed(const Dims& d, const LaunchArgs& a, const AdjArgs& b, const cplx* rho_T, int obs_id,
                         double dAdamp, double dAdomega, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_seed<NB>, dim3(1), dim3(256), 0, st, d, (const cplx*)a.hop, rho_T, a.Ax, a.Ay, a.polx,
                       a.poly, obs_id, b.rhobar, dAdamp, dAdomega, b.theta_bar);
    return hipGetLastError();
  }
};

#define KBE_ADJ_DISPATCH(NBV, CALL)       \
  switch (NBV) {                          \
    case 1: return AdjLaunch<1>::CALL;    \
    case 2: return AdjLaunch<2>::CALL;    \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_adj_bulk(const Dims& d, const LaunchArgs& a, const AdjArgs& b, const cplx* Ibar, int m, int mode,
                           const cplx* sig1, const cplx* Ibar1, hipStream_t st) {
  if (mode != ADJ_SUMS && (mode != ADJ_FUSED || !sig1 || !Ibar1)) return hipErrorInvalidValue;
  KBE_ADJ_DISPATCH(d.nb, bulk(d, a, b, Ibar, m, mode, sig1, Ibar1, st));
}
hipError_t launch_adj_row(const Dims& d, const LaunchArgs& a, const AdjArgs& b, const cplx* Ibar, const cplx* Dbar,
                          int m, hipStream_t st) {
  KBE_ADJ_DISPATCH(d.nb, row(d, a, b, Ibar, Dbar, m, st));
}
hipError_t launch_adj_sigma(const Dims& d, const LaunchArgs& a, const AdjArgs& b, int m, int* nblocks,
                            hipStream_t st) {
  KBE_ADJ_DISPATCH(d.nb, sigma(d, a, b, m, nblocks, st));
}
hipError_t launch_adj_update(const Dims& d, const LaunchArgs& a, const AdjArgs& b, int m, int corrector,
                             const cplx* Gbar_hist, const cplx* Gbar_row, const cplx* rho_prev, hipStream_t st) {
  KBE_ADJ_DISPATCH(d.nb, update(d, a, b, m, corrector, Gbar_hist, Gbar_row, rho_prev, st));
}
hipError_t launch_adj_props(const Dims& d, const LaunchArgs& a, const AdjArgs& b, const cplx* hf,
                            hipStream_t st) {
  KBE_ADJ_DISPATCH(d.nb, props(d, a, b, hf, st));
}
hipError_t launch_adj_hf(const Dims& d, const LaunchArgs& a, const AdjArgs& b, const cplx* rho_prev,
                         const cplx* rho_cur, double wb, cplx* rbar_prev, cplx* rbar_cur, double dAdamp,
                         double dAdomega, hipStream_t st) {
  KBE_ADJ_DISPATCH(d.nb, hf(d, a, b, rho_prev, rho_cur, wb, rbar_prev, rbar_cur, dAdamp, dAdomega, st));
}
hipError_t launch_adj_reduce_u(const AdjArgs& b, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_reduce_u, dim3(1), dim3(256), 0, st, (const double*)b.ubar_part, n, b.theta_bar);
  return hipGetLastError();
}
hipError_t launch_adj_seed(const Dims& d, const LaunchArgs& a, const AdjArgs& b, const cplx* rho_T, int obs_id,
                           double dAdamp, double dAdomega, hipStream_t st) {
  KBE_ADJ_DISPATCH(d.nb, seed(d, a, b, rho_T, obs_id, dAdamp, dAdomega, st));
}

hipError_t launch_adj_rho(const Dims& d, const void* hist, int m, cplx* rho, hipStream_t st) {
  KBE_ADJ_DISPATCH(d.nb, rho(d, hist, m, rho, st));
}

}  // namespace kbe
