// Launch interface of the adjoint (reverse-mode) kernels of the propagation step.
#pragma once
#include "kbe_kernels.hpp"

namespace kbe {

// Device buffers of one reverse sweep. Row buffers are [k][C][Tp] (like the collision rows);
// per-k matrices [k][nb^2]. Adjoints follow the convention  xbar = dL/dRe(x) + i dL/dIm(x)
// for a real loss L.
struct AdjArgs {
  cplx* lam;          // adjoint history: same strip-major layout as the FP64 history
  cplx* Ibar;         // adjoint of the collision row being reversed (eval pass of t_m)
  cplx* Ibar_prev;    // adjoint of I(t_{m-1}, .) being accumulated
  cplx* Ibar_c;       // adjoint of the corrector pass's collision row
  cplx* Rbar;         // adjoint of the current row from a collision-adjoint pass
  cplx* sbar;         // [k][2][nb^2][Tp] adjoint of the Sigma row (lesser, greater)
  cplx* sbar_col;     // [k][C][Tp] per-column Sigma adjoint from the history sums
  cplx* sbar_rowpart; // [k][Smax][nb^2][Tp] per-strip partial adjoint of Sigma^R
  cplx* Dbar;         // adjoint of D of the pass being reversed
  cplx* Dbar_prev;    // adjoint of D_{m-1}
  cplx* Dbar_c;       // adjoint of the corrector pass's D
  cplx* rhobar;       // adjoint of rho_m
  cplx* rhobar_prev;  // adjoint of rho_{m-1}
  cplx* rhobar_P;     // adjoint of the predictor's rho_m
  cplx* props_p;      // recomputed predictor propagators [k][3][nb^2]
  cplx* props_c;      // recomputed corrector propagators
  cplx* pbar;         // [k][3][nb^2] adjoints of V, Vh, Phi
  cplx* rhoP;         // recomputed predictor rho_m
  cplx* Ire_prev;     // recomputed I(t_{m-1}, .)
  cplx* Ire_c;        // recomputed corrector I(t_m, .)
  cplx* Dc;           // recomputed corrector D
  cplx* Dscratch;     // D_{m-1} from the recomputed evaluation pass of t_{m-1}
  cplx* rho0;         // rho_{m-1} (rho_T at the seed) read back from the history diagonal
  cplx* hf_p;         // recomputed predictor mean field [nb^2]
  cplx* hf_c;         // recomputed corrector mean field
  double* kpart;      // [k][NB + 1] per-k partials: dL/dhf_aa, dL/dA
  double* ubar_part;  // per-block partials of dL/dU from the self-energy adjoint
  double* theta_bar;  // [3] dL/d(amp, omega, U)
};

// Modes of the adjoint history sums. A reverse step reverses two collision passes whose history
// sums read the same stored blocks; the adjoint-history update of each is linear in its own
// (Sigma row, Ibar), so the first of them (in reverse order) leaves it to the second:
//   ADJ_SUMS   Sigma adjoints only (reads the history, not the adjoint history)
//   ADJ_FUSED  Sigma adjoints of this pass; adjoint-history update of this pass plus that of the
//              earlier ADJ_SUMS pass, whose Sigma row and Ibar are sig1, Ibar1
// Any other mode, or ADJ_FUSED without sig1 and Ibar1, returns hipErrorInvalidValue.
enum { ADJ_SUMS = 1, ADJ_FUSED = 2 };
hipError_t launch_adj_bulk(const Dims& d, const LaunchArgs& a, const AdjArgs& b, const cplx* Ibar, int m, int mode,
                           const cplx* sig1, const cplx* Ibar1, hipStream_t st);
hipError_t launch_adj_row(const Dims& d, const LaunchArgs& a, const AdjArgs& b, const cplx* Ibar,
                          const cplx* Dbar, int m, hipStream_t st);
hipError_t launch_adj_sigma(const Dims& d, const LaunchArgs& a, const AdjArgs& b, int m, int* nblocks,
                            hipStream_t st);
hipError_t launch_adj_update(const Dims& d, const LaunchArgs& a, const AdjArgs& b, int m, int corrector,
                             const cplx* Gbar_hist, const cplx* Gbar_row, const cplx* rho_prev,
                             hipStream_t st);
hipError_t launch_adj_props(const Dims& d, const LaunchArgs& a, const AdjArgs& b, const cplx* hf,
                            hipStream_t st);
hipError_t launch_adj_hf(const Dims& d, const LaunchArgs& a, const AdjArgs& b, const cplx* rho_prev,
                         const cplx* rho_cur, double wb, cplx* rbar_prev, cplx* rbar_cur, double dAdamp,
                         double dAdomega, hipStream_t st);
hipError_t launch_adj_reduce_u(const AdjArgs& b, int n, hipStream_t st);
// rho[k][nb^2] = rho_m of the committed FP64 history (its diagonal block G^< = i rho_m)
hipError_t launch_adj_rho(const Dims& d, const void* hist, int m, cplx* rho, hipStream_t st);
hipError_t launch_adj_seed(const Dims& d, const LaunchArgs& a, const AdjArgs& b, const cplx* rho_T, int obs_id,
                           double dAdamp, double dAdomega, hipStream_t st);

}  // namespace kbe
