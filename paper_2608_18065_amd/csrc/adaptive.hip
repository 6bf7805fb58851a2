// Adaptive regularisation around the minSR solve:
//   - the Frobenius norm of T and the schedule lambda = c ||T||^{2/3}
//     (Sec. 3.3);
//   - tau = e' - lambda x (Cholesky) or T x (pseudo-inverse), the
//     trust-region rate eta* = eta / ||tau||_2 (App. F), applied by scaling
//     x by eta* / eta before the update forms eta O' x;
//   - the Levenberg-Marquardt ratio of measured to predicted energy
//     decrease and the damping of the next step (App. G).
// Every reduction runs in a fixed order, so the results are reproducible.
// The scalars travel between kernels in a small device report:
//   [0] ||T||_F  [1] lambda used  [2] ||tau||_2  [3] eta used  [4] e'^T tau
//   [5] E_trial  [6] rho  [7] lambda for the next step
#include "model.hpp"

namespace minsr {

// part[b] = sum of T[r][j]^2 over the rows r = b, b + gridDim.x, ...
template <typename TT>
__global__ __launch_bounds__(256) void k_frob_part(const TT* T, int n, double* part) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  double acc = 0.0;
  for (int r = blockIdx.x; r < n; r += gridDim.x)
    for (int j = t; j < n; j += 256) {
      const double v = (double)T[(size_t)r * n + j];
      acc = fma(v, v, acc);
    }
  red[t] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) part[blockIdx.x] = red[0];
}

// report[0] = ||T||_F (parts summed in order); report[1] = the shift:
// lambda (constant), lambda ||T||_F^{2/3} (schedule) or the carried damping
__global__ void k_adapt_lambda(const double* part, int np, int mode, double lambda,
                               const double* carried, double* report) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < np; ++b) s += part[b];
  const double tn = sqrt(s);
  double lu = lambda;
  if (mode == MINSR_LAMBDA_POW23) lu = lambda * pow(tn, 2.0 / 3.0);
  else if (mode == MINSR_LAMBDA_LM) lu = carried[0];
  report[0] = tn;
  report[1] = lu;
  report[5] = 0.0;
  report[6] = 0.0;
  report[7] = 0.0;
}

// y = T x, one wavefront per row (terms in order of j within a lane, lanes
// combined by a fixed tree)
__global__ __launch_bounds__(256) void k_gemv_rows(const double* T, int n, const double* x,
                                                   double* y) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  double acc = 0.0;
  for (int j = lane; j < n; j += 64) acc = fma(T[(size_t)row * n + j], x[j], acc);
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
  if (lane == 0) y[row] = acc;
}

// tau (Cholesky: e' - lambda x with the shift the solve used, report[1];
// pseudo-inverse: T x, computed before), ||tau||_2, e'^T tau, the rate
// (eta / ||tau||_2 with the trust region, else eta), then x *= rate / eta
__global__ __launch_bounds__(1024) void k_tau_final(int n, const double* ep, double* x,
                                                    double* tau, int pinv, double eta, int trust,
                                                    double* report) {
  __shared__ double r2[1024], re[1024];
  const int t = threadIdx.x;
  const double lam = report[1];
  double s2 = 0.0, se = 0.0;
  for (int i = t; i < n; i += 1024) {
    double ti;
    if (pinv) {
      ti = tau[i];
    } else {
      ti = ep[i] - lam * x[i];
      tau[i] = ti;
    }
    s2 = fma(ti, ti, s2);
    se = fma(ep[i], ti, se);
  }
  r2[t] = s2;
  re[t] = se;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if (t < w) { r2[t] += r2[t + w]; re[t] += re[t + w]; }
    __syncthreads();
  }
  const double tn = sqrt(r2[0]);
  const double eu = trust ? eta / tn : eta;
  if (t == 0) {
    report[2] = tn;
    report[3] = eu;
    report[4] = re[0];
  }
  const double sc = eu / eta;
  for (int i = t; i < n; i += 1024) x[i] *= sc;
}

// restore == 0: bak = theta, theta -= dtheta; restore == 1: theta = bak
__global__ void k_trial_theta(double* theta, double* bak, const double* dth, size_t Np,
                              int restore) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Np) return;
  if (restore) {
    theta[k] = bak[k];
  } else {
    const double v = theta[k];
    bak[k] = v;
    theta[k] = v - dth[k];
  }
}

// App. G: rho = (E - E_trial) / (eta_u e'^T tau - eta_u^2 ||tau||^2 / 2)
// and the damping of the next step (omega lambda when rho < 1/4 or is not a
// number, lambda / omega when rho > 3/4)
__global__ void k_lm(const double* E0, const double* E1, double omega, double* carried,
                     double* report) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double tn = report[2], eu = report[3], et = report[4], lam = report[1];
  const double pred = eu * et - 0.5 * eu * eu * (tn * tn);
  const double rho = (E0[0] - E1[0]) / pred;
  double next = lam;
  if (!(rho >= 0.25)) next = omega * lam;
  else if (rho > 0.75) next = lam / omega;
  report[5] = E1[0];
  report[6] = rho;
  report[7] = next;
  carried[0] = next;
}

int launch_adapt_lambda(int n, const void* T, int t_f32, int mode, double lambda,
                        const double* carried, double* part, double* report, hipStream_t s) {
  const int np = std::max(1, std::min(ADAPT_FROB_PARTS, n));
  if (n > 0) {
    if (t_f32) k_frob_part<float><<<np, 256, 0, s>>>((const float*)T, n, part);
    else k_frob_part<double><<<np, 256, 0, s>>>((const double*)T, n, part);
    MINSR_CHECK_LAUNCH();
  }
  k_adapt_lambda<<<1, 64, 0, s>>>(part, n > 0 ? np : 0, mode, lambda, carried, report);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

int launch_tau(int n, const double* T, const double* ep, double* x, double* tau, int pinv,
               double eta, int trust, double* report, hipStream_t s) {
  if (pinv && n > 0) {
    k_gemv_rows<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(T, n, x, tau);
    MINSR_CHECK_LAUNCH();
  }
  k_tau_final<<<1, 1024, 0, s>>>(n, ep, x, tau, pinv, eta, trust, report);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

int launch_trial_theta(double* theta, double* bak, const double* dth, size_t Np, int restore,
                       hipStream_t s) {
  k_trial_theta<<<(unsigned)((Np + 255) / 256), 256, 0, s>>>(theta, bak, dth, Np, restore);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

int launch_lm(const double* E0, const double* E1, double omega, double* carried, double* report,
              hipStream_t s) {
  k_lm<<<1, 64, 0, s>>>(E0, E1, omega, carried, report);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

}  // namespace minsr
