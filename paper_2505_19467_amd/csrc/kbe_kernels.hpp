// Host-side launch interface of the gfx950 Kadanoff-Baym kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kbe_device.hpp"

#define KBE_DEV_INT_HUBBARD 0
#define KBE_DEV_INT_INTERBAND 1
#define KBE_DEV_NOBS 17
#define KBE_DEV_OBS_NORB 9
#define KBE_DEV_OBS_NBAND 13

#define KBE_ROW_PREDICT 0
#define KBE_ROW_CORRECT 1
#define KBE_ROW_EVAL 2
// the corrector's update alone, from the I(t_m, .) an EVAL launch has just stored (launch_row
// runs a corrector pass at nb = 4 as EVAL + UPDATE: kernels of two waves per SIMD, where the
// fused one fits one); UPDATE_CHG also writes the row's largest change (tolerance mode)
#define KBE_ROW_UPDATE 3
#define KBE_ROW_UPDATE_CHG 4

namespace kbe {

// Device pointers and scalars a launch needs (the roles *_prev / *_cur are resolved by
// the caller for the current step).
struct LaunchArgs {
  void* hist;      // packed history, FP64 (cplx) or FP32 (float2) elements
  cplx* row64;     // FP64 working copies of history rows m-1 and m
  cplx* sig;
  cplx* I_prev;
  cplx* I_cur;
  cplx* col0;
  cplx* diag;
  cplx* colsum;
  cplx* rowpart;
  cplx* rho_prev;
  cplx* rho_cur;
  cplx* D_prev;
  cplx* D_cur;
  cplx* props;
  cplx* hfbuf;
  cplx* hop;
  double* eig_w;
  cplx* eig_U;
  double* mu;
  double* obs;
  int commit;      // 0: the row kernel writes only the FP64 working row (recomputation)
  double* chg;     // if set, the corrector row kernel writes max |G_new - G_old| per (k, t') here ([k][Tp])
  cplx* gR;        // interband self-energy: real-space lines of row m, [t_j][comp][ab][R] (else null)
  QuadW quad;      // quadrature weights of eq. (CI)
  double Ax, Ay;  // A(t) * pol for the launch at hand
  double polx, poly;  // pulse polarisation
  double dt, U, UU, temp, target, spin;
  int interaction, hf, corr;
};

hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t st);
hipError_t launch_init(const Dims& d, const LaunchArgs& a, hipStream_t st);
hipError_t launch_hf(const Dims& d, const LaunchArgs& a, double wb, hipStream_t st);
hipError_t launch_props(const Dims& d, const LaunchArgs& a, hipStream_t st);
hipError_t launch_sigma(const Dims& d, const LaunchArgs& a, int m, hipStream_t st);
// the paper's direct-sum self-energy (interband preset, chain with even n <= 1024)
hipError_t launch_sigma_direct(const Dims& d, const LaunchArgs& a, int m, hipStream_t st);
// the dipole kick on the completed slice m (nb = 2): the row's copies and rho_cur (and rho_other)
hipError_t launch_kick(const Dims& d, const LaunchArgs& a, int m, double kc, double ks, cplx* rho_other,
                       hipStream_t st);
hipError_t launch_diag_I(const Dims& d, const LaunchArgs& a, int m, hipStream_t st);
hipError_t launch_bulk(const Dims& d, const LaunchArgs& a, int m, hipStream_t st);
// after each history pass at nb = 4 (a no-op otherwise): sums the strips' row partials into slot 0,
// which the row kernels then read alone; not idempotent, so exactly once per history pass
hipError_t launch_rowpart_fold(const Dims& d, const LaunchArgs& a, int m, hipStream_t st);
hipError_t launch_row(const Dims& d, const LaunchArgs& a, int m, int mode, hipStream_t st);
// out[0] = max over k and t' <= m of chg[k][t'] (one block, deterministic)
hipError_t launch_change_max(const Dims& d, const double* chg, int m, double* out, hipStream_t st);
hipError_t launch_obs(const Dims& d, const LaunchArgs& a, int m, double t, double A, hipStream_t st);
hipError_t launch_aux(const Dims& d, const LaunchArgs& a, int m, hipStream_t st);

}  // namespace kbe
