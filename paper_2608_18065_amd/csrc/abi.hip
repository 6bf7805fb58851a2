// C ABI of the minSR library: argument checking, workspace ownership and
// the order in which one iteration of Algorithm 1 enqueues its kernels.
#include "model.hpp"
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

namespace minsr {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

Layout make_layout(int dim, int H, int cplx) {
  Layout L{};
  L.H = H; L.dim = dim; L.cplx = cplx; L.ds = dim == 1 ? 2 : 4;
  size_t o = 0;
  auto take = [&](size_t n) { size_t r = o; o += n; return r; };
  const size_t h = (size_t)H, ds = (size_t)L.ds;
  if (dim == 2) { L.U1 = take(h * h); L.U2 = take(h * h); }
  L.Wu = take(h * (h + ds)); L.bu = take(h);
  L.Wr = take(h * (h + ds)); L.br = take(h);
  L.Wh = take(h * h); L.bh = take(h);
  L.Win = take(h * ds); L.bin = take(h);
  L.U = take(2 * h); L.c = take(2);
  if (cplx) { L.Uphi = take(2 * h); L.cphi = take(2); }
  L.Np = o;
  return L;
}

size_t packed_elems(minsr_model* m);
void bind_work(minsr_model* m);
size_t gram_partial_bytes(int n, size_t Np, int dtype);

template <typename TO>
__global__ void k_vjp(const TO* O, int Ns, int two, size_t Np, const double* g, double scale,
                      double* out) {
  size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= Np) return;
  double s = 0.0;
  for (int r = 0; r < Ns; ++r) s += g[2 * r] * (double)O[(size_t)r * Np + col];
  if (two)
    for (int r = 0; r < Ns; ++r) s += g[2 * r + 1] * (double)O[((size_t)Ns + r) * Np + col];
  out[col] = s * scale;
}

__global__ void k_widen(const float* a, size_t n, double* out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)a[i];
}

static int alloc(void** p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(MINSR_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return MINSR_OK;
}

// the pseudo-inverse workspace, allocated once per handle (not inside a
// stream capture)
static int ensure_pinv_ws(minsr_model* m, hipStream_t s) {
  if (m->eig) return MINSR_OK;
  const int rows = (m->cplx ? 2 : 1) * m->d.max_Ns;
  const int nmax = std::min(rows, 4096);
  if (s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return fail(MINSR_E_UNSUPPORTED,
                  "pseudo-inverse workspace not reserved: create the model with MINSR_OPT_PINV "
                  "or run one uncaptured pseudo-inverse call first");
  }
  const size_t e = pinv_workspace_doubles(nmax);
  int rc = alloc((void**)&m->eig, e * 8);
  if (rc) return rc;
  m->eig_elems = e;
  m->eig_nmax = nmax;
  return MINSR_OK;
}

static void release(minsr_model* m) {
  void* ptrs[] = {m->theta, m->work, m->nbr, m->subA, m->bonds, m->states, m->gates, m->jdp, m->jtape, m->site,
                  m->contrib,
                  m->elist, m->ecount, m->eitems, m->eloc_q,
                  m->diag, m->ring, m->sigma, m->logpsi, m->eloc, m->stats, m->O, m->R,
                  m->colpart, m->colmean, m->T, m->Lf, m->Dinv, m->gpart, m->epsp, m->x, m->vwork,
                  m->dpart, m->dtheta, m->status, m->eig, m->csync, m->adapt,
                  m->theta_bak};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (hipEvent_t e : m->ev) (void)hipEventDestroy(e);
  m->ev.clear();
}

}  // namespace minsr

using namespace minsr;

extern "C" {

const char* minsr_last_error(void) { return g_err.c_str(); }

int minsr_create_model(const minsr_model_desc* d, minsr_model** out) {
  if (!d || !out) return fail(MINSR_E_INVALID_ARG, "null argument");
  *out = nullptr;
  if (d->dim != 1 && d->dim != 2) return fail(MINSR_E_INVALID_ARG, "dim must be 1 or 2");
  const int H = d->hidden;
  const bool linear = (d->options & MINSR_OPT_LINEAR) != 0;
  if (H != 8 && H != 16 && H != 32 && H != 64 && H != 128)
    return fail(MINSR_E_UNSUPPORTED, "hidden width must be 8, 16, 32, 64 or 128");
  if (linear) {
    if (d->dim != 1 || d->Ly != 1 || d->complex_head || d->marshall || d->zero_mag)
      return fail(MINSR_E_INVALID_ARG, "the linear test model is a real 1D chain without "
                                       "phase head, Marshall sign or S^z mask");
    if (d->compute_dtype != MINSR_F64)
      return fail(MINSR_E_INVALID_ARG, "the linear test model computes in FP64");
    if (H > 64) return fail(MINSR_E_UNSUPPORTED, "linear test model: hidden width at most 64");
  }
  if (d->Lx < 2 || d->Ly < 1) return fail(MINSR_E_INVALID_ARG, "lattice too small");
  if (d->dim == 1 && d->Ly != 1) return fail(MINSR_E_INVALID_ARG, "1D models need Ly == 1");
  if (d->dim == 2 && (d->Ly < 2 || d->Lx > 16))
    return fail(MINSR_E_UNSUPPORTED, "2D models need Ly >= 2 and Lx <= 16");
  const int N = d->Lx * d->Ly;
  if (N > 1024) return fail(MINSR_E_UNSUPPORTED, "at most 1024 sites");
  if (d->zero_mag && (N % 2)) return fail(MINSR_E_INVALID_ARG, "zero_mag needs an even N");
  if (d->compute_dtype != MINSR_F64 && d->compute_dtype != MINSR_F32)
    return fail(MINSR_E_INVALID_ARG, "compute_dtype must be MINSR_F64 or MINSR_F32");
  if (d->max_Ns < 1 || d->max_Ns > (1 << 16)) return fail(MINSR_E_INVALID_ARG, "max_Ns out of range");
  if (d->options & ~(MINSR_OPT_PINV | MINSR_OPT_LINEAR))
    return fail(MINSR_E_INVALID_ARG, "unknown option bits");

  minsr_model* m = new (std::nothrow) minsr_model();
  if (!m) return fail(MINSR_E_NOMEM, "host allocation failed");
  m->d = *d;
  m->N = N; m->H = H; m->dim = d->dim; m->cplx = d->complex_head ? 1 : 0;
  m->ds = d->dim == 1 ? 2 : 4;
  m->f64 = d->compute_dtype == MINSR_F64;
  m->linear = linear ? 1 : 0;
  m->L = make_layout(m->dim, H, m->cplx);
  if (linear) {
    m->L = Layout{};
    m->L.H = H; m->L.ds = 2; m->L.dim = 1;
    m->L.Np = linear_num_params(H);
  }
  if (hipGetDevice(&m->device) != hipSuccess) { delete m; return fail(MINSR_E_DEVICE, "no HIP device"); }

  const size_t Np = m->L.Np, S = (size_t)d->max_Ns, Nz = (size_t)N, Hz = (size_t)H;
  const size_t sz = m->f64 ? 8 : 4;

  // lattice tables: zigzag path predecessors, Marshall sublattice, bonds
  std::vector<int> nbr(2 * N, -1);
  std::vector<uint8_t> subA(N, 0);
  auto pidx = [&](int i, int j) { return j * d->Lx + ((j % 2 == 0) ? i : d->Lx - 1 - i); };
  for (int k = 0; k < N; ++k) {
    const int j = k / d->Lx;
    const int i = (j % 2 == 0) ? k % d->Lx : d->Lx - 1 - k % d->Lx;
    if (m->dim == 2) {
      const int ih = (j % 2 == 0) ? i - 1 : i + 1;
      nbr[2 * k] = (ih >= 0 && ih < d->Lx) ? pidx(ih, j) : -1;
      nbr[2 * k + 1] = j >= 1 ? pidx(i, j - 1) : -1;
    } else {
      nbr[2 * k] = k - 1;
    }
    subA[k] = ((i + j) % 2 == 0) ? 1 : 0;
  }
  std::vector<int> bonds;
  if (m->dim == 2) {
    auto addb = [&](int a, int b) { bonds.push_back(std::min(a, b)); bonds.push_back(std::max(a, b)); };
    for (int j = 0; j < d->Ly; ++j)
      for (int i = 0; i < d->Lx; ++i) {
        if (i + 1 < d->Lx) addb(pidx(i, j), pidx(i + 1, j));
        if (j + 1 < d->Ly) addb(pidx(i, j), pidx(i, j + 1));
      }
    m->n_nn = (int)bonds.size() / 2;
    for (int j = 0; j < d->Ly; ++j)
      for (int i = 0; i < d->Lx; ++i) {
        if (i + 1 < d->Lx && j + 1 < d->Ly) addb(pidx(i, j), pidx(i + 1, j + 1));
        if (i - 1 >= 0 && j + 1 < d->Ly) addb(pidx(i, j), pidx(i - 1, j + 1));
      }
    m->n_nnn = (int)bonds.size() / 2 - m->n_nn;
  }
  m->max_terms = std::max(N, m->n_nn + m->n_nnn);

  const size_t rows = (m->cplx ? 2 : 1) * S;
  const size_t nrc = (S + 31) / 32;
  size_t gp = 0;
  for (int dt : {MINSR_BF16, MINSR_F32, MINSR_F64})
    gp = std::max(gp, gram_partial_bytes((int)rows, Np, dt));
  m->gpart_elems = gp / sizeof(float) + 1;

  int rc = MINSR_OK;
  rc = rc ? rc : alloc((void**)&m->theta, Np * 8);
  size_t pk = linear ? 1 : packed_elems(m);
  m->work_elems = pk;
  rc = rc ? rc : alloc(&m->work, pk * sz);
  rc = rc ? rc : alloc((void**)&m->nbr, nbr.size() * sizeof(int));
  rc = rc ? rc : alloc((void**)&m->subA, subA.size());
  rc = rc ? rc : alloc((void**)&m->bonds, std::max<size_t>(bonds.size(), 2) * sizeof(int));
  rc = rc ? rc : alloc(&m->states, S * Nz * Hz * sz);
  // the Jacobian of these models reads the sampler's gate values instead of
  // recomputing them (checkpoint stride 1)
  if (m->dim == 1 && !m->f64 && m->H <= 64) {
    rc = rc ? rc : alloc(&m->gates, S * Nz * 4 * Hz * sz);
    if (m->H >= 32) rc = rc ? rc : alloc(&m->jdp, (m->cplx ? 2 : 1) * S * Nz * 3 * Hz * sz);
  }
  if (const size_t te = jac_mfma_tape_elems(m->dim, m->f64, m->H, m->N, m->cplx, S))
    rc = rc ? rc : alloc(&m->jtape, te * sizeof(float));
  rc = rc ? rc : alloc((void**)&m->site, S * Nz * 4 * 8);
  rc = rc ? rc : alloc((void**)&m->contrib, (size_t)m->max_terms * S * 2 * 8);
  rc = rc ? rc : alloc((void**)&m->elist, (size_t)m->max_terms * S * 4);
  rc = rc ? rc : alloc((void**)&m->ecount, ((size_t)m->max_terms + 1) * 4);
  rc = rc ? rc : alloc((void**)&m->eitems, (size_t)m->max_terms * ((S + 31) / 32) * 2 * 4);
  if (m->dim == 2) {
    // recompute windows: one per sample (sampling) or per in-flight
    // local-energy sequence (persistent grid of up to 512 x 32 sequences)
    m->ring_blocks = (int)std::max<size_t>(S, 512 * 32);
    rc = rc ? rc : alloc(&m->ring, (size_t)m->ring_blocks * (size_t)(2 * d->Lx) * Hz * sz);
  }
  rc = rc ? rc : alloc((void**)&m->sigma, S * Nz);
  rc = rc ? rc : alloc((void**)&m->logpsi, S * 2 * 8);
  rc = rc ? rc : alloc((void**)&m->eloc, S * 2 * 8);
  rc = rc ? rc : alloc((void**)&m->stats, 4 * 8);
  rc = rc ? rc : alloc(&m->O, rows * Np * sz);
  rc = rc ? rc : alloc(&m->R, rows * padded_ld(Np) * sz);
  rc = rc ? rc : alloc((void**)&m->colpart, 2 * nrc * Np * 8);
  rc = rc ? rc : alloc((void**)&m->colmean, 2 * Np * 8);
  rc = rc ? rc : alloc((void**)&m->T, rows * rows * 8);
  rc = rc ? rc : alloc((void**)&m->Lf, rows * rows * 8);
  rc = rc ? rc : alloc((void**)&m->Dinv, chol_dinv_elems((int)rows) * 8);
  rc = rc ? rc : alloc((void**)&m->gpart, m->gpart_elems * sizeof(float));
  rc = rc ? rc : alloc((void**)&m->epsp, rows * 8);
  rc = rc ? rc : alloc((void**)&m->x, rows * 8);
  rc = rc ? rc : alloc((void**)&m->vwork, chol_vec_elems((int)rows) * 8);
  rc = rc ? rc : alloc((void**)&m->csync, chol_sync_words((int)rows) * 4);
  rc = rc ? rc : alloc((void**)&m->dpart, ((rows + 63) / 64) * Np * 8);
  rc = rc ? rc : alloc((void**)&m->dtheta, Np * 8);
  rc = rc ? rc : alloc((void**)&m->adapt, (rows + 16 + ADAPT_FROB_PARTS) * 8);
  rc = rc ? rc : alloc((void**)&m->theta_bak, Np * 8);
  rc = rc ? rc : alloc((void**)&m->status, 16);
  rc = rc ? rc : alloc((void**)&m->eloc_q, 16);
  if (!rc && (d->options & MINSR_OPT_PINV)) rc = ensure_pinv_ws(m, nullptr);
  if (rc) { release(m); delete m; return rc; }

  hipError_t e = hipMemcpy(m->nbr, nbr.data(), nbr.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->subA, subA.data(), subA.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !bonds.empty())
    e = hipMemcpy(m->bonds, bonds.data(), bonds.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->eloc_q, 0, 16);
  if (e != hipSuccess) { release(m); delete m; return fail(MINSR_E_DEVICE, hipGetErrorString(e)); }
  if (linear) {
    rc = launch_linear_init(m, nullptr);
  } else {
    bind_work(m);
    rc = launch_init_theta(m, nullptr);
    if (!rc) rc = launch_pack(m, nullptr);
  }
  if (!rc && hipDeviceSynchronize() != hipSuccess) rc = fail(MINSR_E_DEVICE, "initialisation failed");
  if (rc) { release(m); delete m; return rc; }
  *out = m;
  return MINSR_OK;
}

int minsr_destroy_model(minsr_model* m) {
  if (!m) return fail(MINSR_E_INVALID_ARG, "null model");
  (void)hipDeviceSynchronize();
  release(m);
  delete m;
  return MINSR_OK;
}

int minsr_num_params(const minsr_model* m, size_t* np) {
  if (!m || !np) return fail(MINSR_E_INVALID_ARG, "null argument");
  *np = m->L.Np;
  return MINSR_OK;
}

int minsr_num_sites(const minsr_model* m, int* n) {
  if (!m || !n) return fail(MINSR_E_INVALID_ARG, "null argument");
  *n = m->N;
  return MINSR_OK;
}

int minsr_get_params(minsr_model* m, double* dev_theta, hipStream_t s) {
  if (!m || !dev_theta) return fail(MINSR_E_INVALID_ARG, "null argument");
  MINSR_HIP(hipMemcpyAsync(dev_theta, m->theta, m->L.Np * 8, hipMemcpyDeviceToDevice, s));
  return MINSR_OK;
}

int minsr_set_params(minsr_model* m, const double* dev_theta, hipStream_t s) {
  if (!m || !dev_theta) return fail(MINSR_E_INVALID_ARG, "null argument");
  MINSR_HIP(hipMemcpyAsync(m->theta, dev_theta, m->L.Np * 8, hipMemcpyDeviceToDevice, s));
  return m->linear ? MINSR_OK : launch_pack(m, s);   // the linear model reads theta itself
}

static int check_ns(minsr_model* m, int Ns) {
  if (!m) return fail(MINSR_E_INVALID_ARG, "null model");
  if (Ns < 0 || Ns > m->d.max_Ns)
    return fail(MINSR_E_SHAPE, "Ns=" + std::to_string(Ns) + " outside [0, max_Ns=" +
                                   std::to_string(m->d.max_Ns) + "]");
  return MINSR_OK;
}

int minsr_sample(minsr_model* m, int Ns, const double* dev_uniforms, uint64_t key,
                 uint64_t counter, uint8_t* dev_sigma, double* dev_logpsi, hipStream_t s) {
  int rc = check_ns(m, Ns);
  if (rc) return rc;
  if (!dev_sigma || !dev_logpsi) return fail(MINSR_E_INVALID_ARG, "null output");
  if (m->linear)
    return launch_linear_forward(m, 0, Ns, dev_uniforms, key, counter, dev_sigma, dev_logpsi, s);
  return launch_forward(m, 0, Ns, dev_uniforms, key, counter, dev_sigma, dev_logpsi, m->states, 1,
                        m->site, s);
}

int minsr_logpsi(minsr_model* m, int Ns, const uint8_t* dev_sigma, double* dev_logpsi,
                 hipStream_t s) {
  int rc = check_ns(m, Ns);
  if (rc) return rc;
  if (!dev_sigma || !dev_logpsi) return fail(MINSR_E_INVALID_ARG, "null argument");
  if (m->linear)
    return launch_linear_forward(m, 1, Ns, nullptr, 0, 0, const_cast<uint8_t*>(dev_sigma),
                                 dev_logpsi, s);
  return launch_forward(m, 1, Ns, nullptr, 0, 0, const_cast<uint8_t*>(dev_sigma), dev_logpsi,
                        m->states, 1, m->site, s);
}

static int check_ham(minsr_model* m, const minsr_hamiltonian* H) {
  if (m->linear) return fail(MINSR_E_UNSUPPORTED, "the linear test model has no local energies");
  if (!H) return fail(MINSR_E_INVALID_ARG, "null Hamiltonian");
  if (H->kind == MINSR_HAM_TFIM || H->kind == MINSR_HAM_CLUSTER) {
    if (m->dim != 1) return fail(MINSR_E_UNSUPPORTED, "TFIM / cluster need a 1D model");
    if (H->kind == MINSR_HAM_CLUSTER && m->N < 3) return fail(MINSR_E_SHAPE, "cluster needs N >= 3");
    return MINSR_OK;
  }
  if (H->kind == MINSR_HAM_J1J2) {
    if (m->dim != 2) return fail(MINSR_E_UNSUPPORTED, "J1-J2 needs a 2D model");
    return MINSR_OK;
  }
  return fail(MINSR_E_INVALID_ARG, "unknown Hamiltonian kind");
}

int minsr_local_energy(minsr_model* m, const minsr_hamiltonian* H, int Ns,
                       const uint8_t* dev_sigma, const double* dev_logpsi, double* dev_eloc,
                       double* dev_stats, hipStream_t s) {
  int rc = check_ns(m, Ns);
  if (rc) return rc;
  if ((rc = check_ham(m, H))) return rc;
  if (!dev_sigma || !dev_eloc) return fail(MINSR_E_INVALID_ARG, "null argument");
  // hidden states and per-site conditionals of the given configurations
  rc = launch_forward(m, 1, Ns, nullptr, 0, 0, const_cast<uint8_t*>(dev_sigma), m->logpsi,
                      m->states, 1, m->site, s);
  if (rc) return rc;
  rc = launch_eloc(m, H, Ns, dev_sigma, dev_logpsi, m->states, m->site, dev_eloc, s);
  if (rc) return rc;
  if (dev_stats) rc = launch_stats(m, Ns, dev_eloc, dev_stats, nullptr, nullptr, s);
  return rc;
}

int minsr_jacobian(minsr_model* m, int Ns, const uint8_t* dev_sigma, int out_dtype, int centered,
                   int ckpt_every, void* dev_O, double* dev_colmean, hipStream_t s) {
  int rc = check_ns(m, Ns);
  if (rc) return rc;
  if (!dev_sigma || !dev_O) return fail(MINSR_E_INVALID_ARG, "null argument");
  if (out_dtype != MINSR_F64 && out_dtype != MINSR_F32 && out_dtype != MINSR_BF16)
    return fail(MINSR_E_INVALID_ARG, "unknown out_dtype");
  if (out_dtype == MINSR_BF16 && !centered)
    return fail(MINSR_E_INVALID_ARG, "BF16 output requires centred rows");
  if (ckpt_every < 1 || ckpt_every > 16) return fail(MINSR_E_INVALID_ARG, "ckpt_every in [1, 16]");
  if (centered && !dev_colmean) return fail(MINSR_E_INVALID_ARG, "centred output needs dev_colmean");
  if (m->linear) {
    rc = launch_linear_forward(m, 1, Ns, nullptr, 0, 0, const_cast<uint8_t*>(dev_sigma),
                               m->logpsi, s);
    if (rc) return rc;
    if (!centered && out_dtype == MINSR_F64)
      return launch_linear_jacobian(m, Ns, dev_sigma, (double*)dev_O, s);
    rc = launch_linear_jacobian(m, Ns, dev_sigma, (double*)m->O, s);
    if (rc) return rc;
    return launch_center(Ns, 1, m->L.Np, m->O, 1, dev_O, out_dtype, m->colpart,
                         centered ? dev_colmean : nullptr, m->L.Np, s);
  }
  const int C = m->dim == 1 ? ckpt_every : 1;
  void* tape = C == 1 ? m->gates : nullptr;
  double* site = m->site;   // the pass's per-site conditionals
  rc = launch_forward(m, 1, Ns, nullptr, 0, 0, const_cast<uint8_t*>(dev_sigma), m->logpsi,
                      m->states, C, site, s, nullptr, tape);
  if (rc) return rc;
  const int native = m->f64 ? MINSR_F64 : MINSR_F32;
  const int nb = m->cplx ? 2 : 1;
  if (!centered && out_dtype == native)
    return launch_jacobian(m, Ns, dev_sigma, m->states, C, dev_O, nullptr, nullptr, s, tape,
                           site);
  rc = launch_jacobian(m, Ns, dev_sigma, m->states, C, m->O, nullptr, nullptr, s, tape, site);
  if (rc) return rc;
  return launch_center(Ns, nb, m->L.Np, m->O, m->f64, dev_O, out_dtype, m->colpart,
                       centered ? dev_colmean : nullptr, m->L.Np, s);
}

int minsr_logpsi_vjp(minsr_model* m, int Ns, const uint8_t* dev_sigma, const double* dev_g,
                     double* dev_grad_theta, hipStream_t s) {
  int rc = check_ns(m, Ns);
  if (rc) return rc;
  if (!dev_sigma || !dev_g || !dev_grad_theta) return fail(MINSR_E_INVALID_ARG, "null argument");
  if (m->linear) return fail(MINSR_E_UNSUPPORTED, "vjp: not for the linear test model");
  if (Ns == 0) {
    MINSR_HIP(hipMemsetAsync(dev_grad_theta, 0, m->L.Np * 8, s));
    return MINSR_OK;
  }
  rc = launch_forward(m, 1, Ns, nullptr, 0, 0, const_cast<uint8_t*>(dev_sigma), m->logpsi,
                      m->states, 1, m->site, s, nullptr, m->gates);
  if (rc) return rc;
  rc = launch_jacobian(m, Ns, dev_sigma, m->states, 1, m->O, nullptr, nullptr, s, m->gates,
                       m->site);
  if (rc) return rc;
  const size_t Np = m->L.Np;
  const double scale = std::sqrt((double)Ns);
  const unsigned grid = (unsigned)((Np + 255) / 256);
  if (m->f64) k_vjp<double><<<grid, 256, 0, s>>>((const double*)m->O, Ns, m->cplx, Np, dev_g, scale, dev_grad_theta);
  else k_vjp<float><<<grid, 256, 0, s>>>((const float*)m->O, Ns, m->cplx, Np, dev_g, scale, dev_grad_theta);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

// the step in three stages (bits of `stages`): 1 = sampling through the
// real form O', 2 = the Gram, 4 = the solve and the update; a batch runs the
// Grams of its instances in one grouped launch between stages 1 and 4
static int step_stages(minsr_model* m, const minsr_hamiltonian* H, const minsr_step_cfg* cfg,
                       const minsr_step_state* st, const minsr_step_out* out, hipStream_t s,
                       int stages) {
  if (!m || !cfg || !st || !out) return fail(MINSR_E_INVALID_ARG, "null argument");
  int rc = check_ns(m, cfg->Ns);
  if (rc) return rc;
  if ((rc = check_ham(m, H))) return rc;
  const int Ns = cfg->Ns;
  if (Ns < 2) return fail(MINSR_E_SHAPE, "a step needs Ns >= 2");
  if (!out->dev_energy || !out->dev_status) return fail(MINSR_E_INVALID_ARG, "null output");
  if (cfg->apply_update && !st->dev_momentum) return fail(MINSR_E_INVALID_ARG, "null momentum");
  if (cfg->form < 0 || cfg->form > 3) return fail(MINSR_E_INVALID_ARG, "unknown form");
  if (!(cfg->lambda >= 0.0) || !(cfg->pinv_cutoff >= 0.0)) return fail(MINSR_E_INVALID_ARG, "negative lambda / cutoff");
  if (cfg->pinv_cutoff == 0.0 && cfg->lambda == 0.0)
    return fail(MINSR_E_INVALID_ARG, "lambda = 0 needs the pseudo-inverse (T is singular)");
  if (cfg->pinv_cutoff > 0.0 && cfg->lambda != 0.0)
    return fail(MINSR_E_INVALID_ARG, "the pseudo-inverse solve takes lambda = 0");
  if (cfg->pinv_cutoff > 0.0 && cfg->form == MINSR_FORM_FP32_PLAIN)
    return fail(MINSR_E_UNSUPPORTED, "the pseudo-inverse solve runs in FP64 only");
  if (cfg->form == MINSR_FORM_FP64_REF && !m->f64)
    return fail(MINSR_E_INVALID_ARG, "the FP64 reference form needs an FP64 model");
  const int C = m->dim == 1 ? cfg->ckpt_every : 1;
  if (C < 1 || C > 16) return fail(MINSR_E_INVALID_ARG, "ckpt_every in [1, 16]");

  const size_t Np = m->L.Np;
  const int nb = m->cplx ? 2 : 1;
  const int n = nb * Ns;
  uint8_t* sigma = out->dev_sigma ? out->dev_sigma : m->sigma;
  double* eloc = out->dev_eloc ? out->dev_eloc : m->eloc;
  double* dth = out->dev_dtheta ? out->dev_dtheta : m->dtheta;
  const int rdt = cfg->form == MINSR_FORM_FP64_REF ? MINSR_F64
                  : cfg->form == MINSR_FORM_FP32_PLAIN ? MINSR_F32 : MINSR_BF16;
  // the hi/lo split keeps both BF16 halves in the O' buffer (rows x ld each)
  void* Rlo = cfg->form == MINSR_FORM_BF16_FP64
                  ? (void*)((__hip_bfloat16*)m->R + (size_t)n * padded_ld(Np))
                  : nullptr;

  const bool timing = m->t_slot < m->t_max;
  auto mark = [&](int phase) -> int {
    if (timing) MINSR_HIP(hipEventRecord(m->ev[(size_t)m->t_slot * (MINSR_NPHASES + 1) + phase], s));
    return MINSR_OK;
  };
#define MINSR_PHASE(ph) do { int rc_ = mark(ph); if (rc_) return rc_; } while (0)

  if (stages & 1) {
  MINSR_PHASE(0);
  // 1. exact autoregressive samples, hidden states, per-site conditionals
  //    (the sampler also clears the status word)
  rc = launch_forward(m, 0, Ns, nullptr, st->key, st->counter, sigma, m->logpsi, m->states, 1,
                      m->site, s, st->dev_counter, C == 1 ? m->gates : nullptr, out->dev_status);
  if (rc) return rc;
  MINSR_PHASE(1);
  // 2. local energies, E, Var and eps'
  rc = launch_eloc(m, H, Ns, sigma, m->logpsi, m->states, m->site, eloc, s, 1);
  if (rc) return rc;
  MINSR_PHASE(2);
  rc = launch_eloc(m, H, Ns, sigma, m->logpsi, m->states, m->site, eloc, s, 2);
  if (rc) return rc;
  rc = launch_stats(m, Ns, eloc, out->dev_energy, m->epsp, out->dev_status, s);
  if (rc) return rc;
  MINSR_PHASE(3);
  // 3. log-derivatives, centring and real form
  rc = launch_jacobian(m, Ns, sigma, m->states, C, m->O, nullptr, nullptr, s,
                       C == 1 ? m->gates : nullptr, m->site);
  if (rc) return rc;
  MINSR_PHASE(4);
  rc = launch_center(Ns, nb, Np, m->O, m->f64, m->R, rdt, m->colpart, m->colmean, padded_ld(Np), s,
                     Rlo);
  if (rc) return rc;
  MINSR_PHASE(5);
  }
  // 4. Gram and regularised solve
  if (stages & 2) {
  rc = launch_gram(n, Np, m->R, rdt, m->T, m->gpart, m->gpart_elems, s, 1, Rlo,
                   m->tune_gram_split);
  if (rc) return rc;
  MINSR_PHASE(6);
  rc = launch_gram(n, Np, m->R, rdt, m->T, m->gpart, m->gpart_elems, s, 2, Rlo,
                   m->tune_gram_split);
  if (rc) return rc;
  MINSR_PHASE(7);
  }
  if (stages & 4) {
  if (cfg->pinv_cutoff > 0.0) {
    rc = ensure_pinv_ws(m, s);
    if (!rc) rc = launch_report_trace(n, m->T, out->dev_tnorm, out->dev_lambda_used, s);
    if (!rc)
      rc = launch_pinv_solve(n, m->T, cfg->pinv_cutoff, m->epsp, m->x, m->eig, m->eig_elems,
                             m->eig_nmax, out->dev_status, s);
  } else {
    // BF16 forms: every entry of T carries FP32 accumulation error of at
    // most about 2^-24 sqrt(T_ii T_jj) (flushes to FP64 every 128 inputs),
    // so its spectral-norm error is below 2^-24 tr T: the shift is kept at
    // least that (measured: a trajectory with tr T = 2.0e6 had a computed T
    // with smallest eigenvalue -0.022, the exact Gram of its operand being
    // positive semidefinite, against 2^-24 tr T = 0.12)
    rc = launch_cholesky_solve(n, m->T, m->Lf, m->Dinv, rdt == MINSR_F32, cfg->lambda, m->epsp,
                               m->x, m->vwork, m->csync, out->dev_status, s,
                               rdt == MINSR_BF16 ? 0x1p-24 : 0.0, out->dev_tnorm,
                               out->dev_lambda_used, nullptr, (uint32_t)m->tune_spin_limit);
  }
  if (rc) return rc;
  MINSR_PHASE(8);
  // 5. dtheta = eta O' x, momentum, parameters, working copy (the update
  //    also advances the device-side Philox counter)
  rc = launch_update(n, Np, m->R, rdt, m->x, cfg->eta, cfg->mu, m->dpart, dth, st->dev_momentum,
                     m->theta, out->dev_status, cfg->apply_update, s, Rlo, st->dev_counter);
  if (rc) return rc;
  MINSR_PHASE(9);
  if (cfg->apply_update) {
    rc = launch_pack(m, s);
    if (rc) return rc;
  }
  MINSR_PHASE(10);
  if (timing) m->t_slot++;
  m->last_n = n;
  m->last_form = cfg->form;
  }
#undef MINSR_PHASE
  return MINSR_OK;
}

int minsr_step(minsr_model* m, const minsr_hamiltonian* H, const minsr_step_cfg* cfg,
               const minsr_step_state* st, const minsr_step_out* out, hipStream_t s) {
  return step_stages(m, H, cfg, st, out, s, 7);
}



int minsr_step_adaptive(minsr_model* m, const minsr_hamiltonian* H, const minsr_step_cfg* cfg,
                        const minsr_adaptive_cfg* ad, const minsr_step_state* st,
                        const minsr_step_out* out, hipStream_t s) {
  if (!m || !cfg || !ad || !st || !out) return fail(MINSR_E_INVALID_ARG, "null argument");
  int rc = check_ns(m, cfg->Ns);
  if (rc) return rc;
  if ((rc = check_ham(m, H))) return rc;
  const int Ns = cfg->Ns;
  if (Ns < 2) return fail(MINSR_E_SHAPE, "a step needs Ns >= 2");
  if (!out->dev_energy || !out->dev_status) return fail(MINSR_E_INVALID_ARG, "null output");
  if (cfg->apply_update && !st->dev_momentum) return fail(MINSR_E_INVALID_ARG, "null momentum");
  if (cfg->form < 0 || cfg->form > 3) return fail(MINSR_E_INVALID_ARG, "unknown form");
  if (cfg->form == MINSR_FORM_FP64_REF && !m->f64)
    return fail(MINSR_E_INVALID_ARG, "the FP64 reference form needs an FP64 model");
  const int mode = ad->lambda_mode;
  if (mode != MINSR_LAMBDA_CONST && mode != MINSR_LAMBDA_POW23 && mode != MINSR_LAMBDA_LM)
    return fail(MINSR_E_INVALID_ARG, "unknown lambda_mode");
  if (ad->trust_region != 0 && ad->trust_region != 1)
    return fail(MINSR_E_INVALID_ARG, "trust_region must be 0 or 1");
  const bool pinv = cfg->pinv_cutoff > 0.0;
  if (!(cfg->pinv_cutoff >= 0.0)) return fail(MINSR_E_INVALID_ARG, "negative cutoff");
  if (pinv) {
    if (mode != MINSR_LAMBDA_CONST || cfg->lambda != 0.0)
      return fail(MINSR_E_INVALID_ARG, "the pseudo-inverse solve takes lambda = 0 (CONST mode)");
    if (cfg->form == MINSR_FORM_FP32_PLAIN)
      return fail(MINSR_E_UNSUPPORTED, "the pseudo-inverse solve runs in FP64 only");
  } else {
    if (mode != MINSR_LAMBDA_LM && !(cfg->lambda > 0.0))
      return fail(MINSR_E_INVALID_ARG, "the Cholesky solve needs lambda > 0");
    if (mode != MINSR_LAMBDA_CONST && cfg->form == MINSR_FORM_FP32_PLAIN)
      return fail(MINSR_E_UNSUPPORTED, "adaptive shifts need an FP64 solve");
  }
  if (mode == MINSR_LAMBDA_LM) {
    if (!ad->dev_lambda) return fail(MINSR_E_INVALID_ARG, "LM mode needs dev_lambda");
    if (st->dev_counter) return fail(MINSR_E_UNSUPPORTED, "LM mode needs a host-side counter");
    if (!(ad->omega > 1.0)) return fail(MINSR_E_INVALID_ARG, "omega must be > 1");
  }
  const int C = m->dim == 1 ? cfg->ckpt_every : 1;
  if (C < 1 || C > 16) return fail(MINSR_E_INVALID_ARG, "ckpt_every in [1, 16]");

  const size_t Np = m->L.Np;
  const int nb = m->cplx ? 2 : 1;
  const int n = nb * Ns;
  uint8_t* sigma = out->dev_sigma ? out->dev_sigma : m->sigma;
  double* eloc = out->dev_eloc ? out->dev_eloc : m->eloc;
  double* dth = out->dev_dtheta ? out->dev_dtheta : m->dtheta;
  const int rdt = cfg->form == MINSR_FORM_FP64_REF ? MINSR_F64
                  : cfg->form == MINSR_FORM_FP32_PLAIN ? MINSR_F32 : MINSR_BF16;
  void* Rlo = cfg->form == MINSR_FORM_BF16_FP64
                  ? (void*)((__hip_bfloat16*)m->R + (size_t)n * padded_ld(Np))
                  : nullptr;
  const size_t rows = (size_t)(m->cplx ? 2 : 1) * m->d.max_Ns;
  double* tau = m->adapt;
  double* report = ad->dev_report ? ad->dev_report : m->adapt + rows;
  double* tstats = m->adapt + rows + 8;
  double* part = m->adapt + rows + 16;

  // 1-4: samples, local energies, E and eps', log-derivative rows, centred
  // real form, T (as minsr_step)
  rc = launch_forward(m, 0, Ns, nullptr, st->key, st->counter, sigma, m->logpsi, m->states, 1,
                      m->site, s, st->dev_counter, C == 1 ? m->gates : nullptr, out->dev_status);
  if (!rc) rc = launch_eloc(m, H, Ns, sigma, m->logpsi, m->states, m->site, eloc, s, 3);
  if (!rc) rc = launch_stats(m, Ns, eloc, out->dev_energy, m->epsp, out->dev_status, s);
  if (!rc) rc = launch_jacobian(m, Ns, sigma, m->states, C, m->O, nullptr, nullptr, s,
                                C == 1 ? m->gates : nullptr, m->site);
  if (!rc) rc = launch_center(Ns, nb, Np, m->O, m->f64, m->R, rdt, m->colpart, m->colmean,
                              padded_ld(Np), s, Rlo);
  if (!rc) rc = launch_gram(n, Np, m->R, rdt, m->T, m->gpart, m->gpart_elems, s, 3, Rlo,
                            m->tune_gram_split);
  if (rc) return rc;
  // ||T||_F and the shift (Sec. 3.3), then the solve; report[1] ends up as
  // the shift the solve used
  rc = launch_adapt_lambda(n, m->T, rdt == MINSR_F32, mode, pinv ? 0.0 : cfg->lambda,
                           ad->dev_lambda, part, report, s);
  if (rc) return rc;
  if (pinv) {
    rc = ensure_pinv_ws(m, s);
    if (!rc) rc = launch_report_trace(n, m->T, out->dev_tnorm, out->dev_lambda_used, s);
    if (!rc)
      rc = launch_pinv_solve(n, m->T, cfg->pinv_cutoff, m->epsp, m->x, m->eig, m->eig_elems,
                             m->eig_nmax, out->dev_status, s);
  } else {
    rc = launch_cholesky_solve(n, m->T, m->Lf, m->Dinv, rdt == MINSR_F32, cfg->lambda, m->epsp,
                               m->x, m->vwork, m->csync, out->dev_status, s,
                               rdt == MINSR_BF16 ? 0x1p-24 : 0.0, out->dev_tnorm, report + 1,
                               mode == MINSR_LAMBDA_CONST ? nullptr : report + 1,
                               (uint32_t)m->tune_spin_limit);
    if (!rc && out->dev_lambda_used)
      rc = hipMemcpyAsync(out->dev_lambda_used, report + 1, 8, hipMemcpyDeviceToDevice, s) ==
                   hipSuccess ? MINSR_OK : fail(MINSR_E_DEVICE, "copy of the shift failed");
  }
  if (rc) return rc;
  // tau, the rate (App. F), x scaled by rate / eta
  rc = launch_tau(n, m->T, m->epsp, m->x, tau, pinv ? 1 : 0, cfg->eta, ad->trust_region,
                  report, s);
  if (rc) return rc;
  if (mode == MINSR_LAMBDA_LM) {
    // dtheta, then the trial energy at theta - dtheta from fresh samples
    // (App. G), with theta restored afterwards
    rc = launch_update(n, Np, m->R, rdt, m->x, cfg->eta, cfg->mu, m->dpart, dth,
                       st->dev_momentum, m->theta, out->dev_status, 0, s, Rlo, nullptr);
    if (!rc) rc = launch_trial_theta(m->theta, m->theta_bak, dth, Np, 0, s);
    if (!rc) rc = launch_pack(m, s);
    if (!rc)
      rc = launch_forward(m, 0, Ns, nullptr, st->key, st->counter ^ (1ull << 63), m->sigma,
                          m->logpsi, m->states, 1, m->site, s);
    if (!rc) rc = launch_eloc(m, H, Ns, m->sigma, m->logpsi, m->states, m->site, m->eloc, s, 3);
    if (!rc) rc = launch_stats(m, Ns, m->eloc, tstats, nullptr, nullptr, s);
    if (!rc) rc = launch_trial_theta(m->theta, m->theta_bak, dth, Np, 1, s);
    if (!rc) rc = launch_pack(m, s);
    if (!rc) rc = launch_lm(out->dev_energy, tstats, ad->omega, ad->dev_lambda, report, s);
    if (rc) return rc;
  }
  // the update (momentum and parameters, App. B) with the scaled x
  rc = launch_update(n, Np, m->R, rdt, m->x, cfg->eta, cfg->mu, m->dpart, dth, st->dev_momentum,
                     m->theta, out->dev_status, cfg->apply_update, s, Rlo, st->dev_counter);
  if (!rc && cfg->apply_update) rc = launch_pack(m, s);
  if (rc) return rc;
  m->last_n = n;
  m->last_form = cfg->form;
  return MINSR_OK;
}

int minsr_timing_begin(minsr_model* m, int max_steps) {
  if (!m || max_steps < 0) return fail(MINSR_E_INVALID_ARG, "bad argument");
  const size_t need = (size_t)max_steps * (MINSR_NPHASES + 1);
  while (m->ev.size() < need) {
    hipEvent_t e;
    MINSR_HIP(hipEventCreate(&e));
    m->ev.push_back(e);
  }
  m->t_max = max_steps;
  m->t_slot = 0;
  return MINSR_OK;
}

int minsr_timing_read(minsr_model* m, double* ms, int* nsteps) {
  if (!m || !ms || !nsteps) return fail(MINSR_E_INVALID_ARG, "null argument");
  for (int p = 0; p < MINSR_NPHASES; ++p) ms[p] = 0.0;
  for (int t = 0; t < m->t_slot; ++t) {
    hipEvent_t* e = &m->ev[(size_t)t * (MINSR_NPHASES + 1)];
    MINSR_HIP(hipEventSynchronize(e[MINSR_NPHASES]));
    for (int p = 0; p < MINSR_NPHASES; ++p) {
      float f = 0.f;
      MINSR_HIP(hipEventElapsedTime(&f, e[p], e[p + 1]));
      ms[p] += f;
    }
  }
  *nsteps = m->t_slot;
  m->t_max = 0;
  m->t_slot = 0;
  return MINSR_OK;
}

int minsr_set_tunable(minsr_model* m, const char* key, int value) {
  if (!m || !key) return fail(MINSR_E_INVALID_ARG, "null argument");
  const std::string k(key);
  if (k == "gram_split") {
    if (value < 0 || value > 64) return fail(MINSR_E_INVALID_ARG, "gram_split in [0, 64]");
    m->tune_gram_split = value;
  } else if (k == "eloc_grid") {
    if (value < 0 || value > (1 << 20)) return fail(MINSR_E_INVALID_ARG, "eloc_grid out of range");
    m->tune_eloc_grid = value;
  } else if (k == "sample_r") {
    if (value != 0 && value != 1 && value != 4) return fail(MINSR_E_INVALID_ARG, "sample_r in {0, 1, 4}");
    m->tune_sample_r = value;
  } else if (k == "jac_parts") {
    if (value != 0 && value != 1 && value != 2 && value != 4)
      return fail(MINSR_E_INVALID_ARG, "jac_parts in {0, 1, 2, 4}");
    m->tune_jac_parts = value;
  } else if (k == "solve_spin_limit") {
    if (value < 0) return fail(MINSR_E_INVALID_ARG, "solve_spin_limit must be >= 0");
    m->tune_spin_limit = value;
  } else {
    return fail(MINSR_E_INVALID_ARG, "unknown tunable " + k);
  }
  return MINSR_OK;
}

int minsr_get_tunable(const minsr_model* m, const char* key, int* value) {
  if (!m || !key || !value) return fail(MINSR_E_INVALID_ARG, "null argument");
  const std::string k(key);
  if (k == "gram_split") *value = m->tune_gram_split;
  else if (k == "eloc_grid") *value = m->tune_eloc_grid;
  else if (k == "sample_r") *value = m->tune_sample_r;
  else if (k == "jac_parts") *value = m->tune_jac_parts;
  else if (k == "solve_spin_limit") *value = m->tune_spin_limit;
  else return fail(MINSR_E_INVALID_ARG, "unknown tunable " + k);
  return MINSR_OK;
}

int minsr_step_intermediates(minsr_model* m, const void** T, const double** x,
                             const double** eps_prime, const void** Oprime, int* n, int* Np) {
  if (!m) return fail(MINSR_E_INVALID_ARG, "null model");
  if (T) *T = m->T;  // the factorisation works on a copy
  if (x) *x = m->x;
  if (eps_prime) *eps_prime = m->epsp;
  if (Oprime) *Oprime = m->R;
  if (n) *n = m->last_n;
  if (Np) *Np = (int)padded_ld(m->L.Np);   // row stride of O' (zero padded)
  return MINSR_OK;
}

int minsr_solve(minsr_model* m, int n, const double* dev_T, double lambda, double pinv_cutoff,
                const double* dev_b, double* dev_x, uint32_t* dev_status, hipStream_t s) {
  if (!m || !dev_T || !dev_b || !dev_x || !dev_status)
    return fail(MINSR_E_INVALID_ARG, "null argument");
  const int rows_max = (m->cplx ? 2 : 1) * m->d.max_Ns;
  if (n < 0 || n > rows_max)
    return fail(MINSR_E_SHAPE, "n = " + std::to_string(n) + " outside [0, " +
                                   std::to_string(rows_max) + "]");
  if (!(lambda >= 0.0) || !(pinv_cutoff >= 0.0))
    return fail(MINSR_E_INVALID_ARG, "negative lambda / cutoff");
  if (pinv_cutoff > 0.0) {
    if (lambda != 0.0) return fail(MINSR_E_INVALID_ARG, "the pseudo-inverse solve takes lambda = 0");
    const int rc = ensure_pinv_ws(m, s);
    if (rc) return rc;
    return launch_pinv_solve(n, const_cast<double*>(dev_T), pinv_cutoff, dev_b, dev_x, m->eig,
                             m->eig_elems, m->eig_nmax, dev_status, s);
  }
  return launch_cholesky_solve(n, dev_T, m->Lf, m->Dinv, 0, lambda, dev_b, dev_x, m->vwork,
                               m->csync, dev_status, s, 0.0, nullptr, nullptr, nullptr,
                               (uint32_t)m->tune_spin_limit);
}

// raw log-derivative rows of the configurations into the handle's O
// (checkpoint stride 1)
static int raw_rows(minsr_model* m, int Ns, const uint8_t* dev_sigma, hipStream_t s) {
  if (m->linear) {
    int rc = launch_linear_forward(m, 1, Ns, nullptr, 0, 0, const_cast<uint8_t*>(dev_sigma),
                                   m->logpsi, s);
    return rc ? rc : launch_linear_jacobian(m, Ns, dev_sigma, (double*)m->O, s);
  }
  void* tape = m->dim == 1 ? m->gates : nullptr;
  int rc = launch_forward(m, 1, Ns, nullptr, 0, 0, const_cast<uint8_t*>(dev_sigma), m->logpsi,
                          m->states, 1, m->site, s, nullptr, tape);
  if (rc) return rc;
  return launch_jacobian(m, Ns, dev_sigma, m->states, 1, m->O, nullptr, nullptr, s, tape, m->site);
}

int minsr_param_gram(minsr_model* m, int Ns, const uint8_t* dev_sigma, double* dev_S,
                     hipStream_t s) {
  int rc = check_ns(m, Ns);
  if (rc) return rc;
  if (!dev_sigma || !dev_S) return fail(MINSR_E_INVALID_ARG, "null argument");
  if (Ns < 1) return fail(MINSR_E_SHAPE, "needs Ns >= 1");
  const size_t Np = m->L.Np;
  const int nb = m->cplx ? 2 : 1;
  // log-derivative rows, centred per block of Ns rows into the real form,
  // then R^T R
  rc = raw_rows(m, Ns, dev_sigma, s);
  if (rc) return rc;
  const int rdt = m->f64 ? MINSR_F64 : MINSR_F32;
  rc = launch_center(Ns, nb, Np, m->O, m->f64, m->R, rdt, m->colpart, m->colmean, padded_ld(Np),
                     s);
  if (rc) return rc;
  return launch_param_gram(m->R, m->f64, nb * Ns, (int)Np, padded_ld(Np), dev_S, s);
}

int minsr_gram(minsr_model* m, int Ns, const uint8_t* dev_sigma, int form, double* dev_T,
               hipStream_t s) {
  int rc = check_ns(m, Ns);
  if (rc) return rc;
  if (!dev_sigma || !dev_T) return fail(MINSR_E_INVALID_ARG, "null argument");
  if (Ns < 1) return fail(MINSR_E_SHAPE, "needs Ns >= 1");
  if (form < 0 || form > 3) return fail(MINSR_E_INVALID_ARG, "unknown form");
  if (form == MINSR_FORM_FP64_REF && !m->f64)
    return fail(MINSR_E_INVALID_ARG, "the FP64 reference form needs an FP64 model");
  const size_t Np = m->L.Np;
  const int nb = m->cplx ? 2 : 1;
  const int n = nb * Ns;
  const int rdt = form == MINSR_FORM_FP64_REF ? MINSR_F64
                  : form == MINSR_FORM_FP32_PLAIN ? MINSR_F32 : MINSR_BF16;
  void* Rlo = form == MINSR_FORM_BF16_FP64
                  ? (void*)((__hip_bfloat16*)m->R + (size_t)n * padded_ld(Np))
                  : nullptr;
  rc = raw_rows(m, Ns, dev_sigma, s);
  if (rc) return rc;
  rc = launch_center(Ns, nb, Np, m->O, m->f64, m->R, rdt, m->colpart, m->colmean, padded_ld(Np), s,
                     Rlo);
  if (rc) return rc;
  // the FP32 form produces an FP32 T in the handle's buffer, widened here
  double* Tout = rdt == MINSR_F32 ? m->T : dev_T;
  rc = launch_gram(n, Np, m->R, rdt, Tout, m->gpart, m->gpart_elems, s, 3, Rlo,
                   m->tune_gram_split);
  if (rc || rdt != MINSR_F32) return rc;
  const size_t nn = (size_t)n * n;
  k_widen<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>((const float*)m->T, nn, dev_T);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

int minsr_spectrum(minsr_model* m, int n, const double* dev_T, double lambda, double eps,
                   double* dev_w, double* dev_cond, uint32_t* dev_status, hipStream_t s) {
  if (!m || !dev_T || !dev_w || !dev_status) return fail(MINSR_E_INVALID_ARG, "null argument");
  const int rows_max = std::min((m->cplx ? 2 : 1) * m->d.max_Ns, 4096);
  if (n < 0 || n > rows_max)
    return fail(MINSR_E_SHAPE, "n = " + std::to_string(n) + " outside [0, " +
                                   std::to_string(rows_max) + "]");
  if (!(lambda >= 0.0) || !(eps > 0.0)) return fail(MINSR_E_INVALID_ARG, "lambda < 0 or eps <= 0");
  const int rc = ensure_pinv_ws(m, s);
  if (rc) return rc;
  return launch_spectrum(n, dev_T, lambda, eps, dev_w, dev_cond, m->eig, m->eig_elems,
                         m->eig_nmax, dev_status, s);
}

// ------------------------------------------------------------------ batch
}  // extern "C"

struct minsr_batch {
  std::vector<minsr_model*> models;
  std::vector<minsr_hamiltonian> hams;
  std::vector<minsr_step_cfg> cfgs;
  std::vector<minsr_step_state> states;
  std::vector<minsr_step_out> outs;
  std::vector<hipStream_t> streams;  // [i] instance i, [count] capture origin
  // [0] fork, [1 + i] join of instance i's first stage; [count + 1] fork of
  // the last stages, [count + 2 + i] their joins
  std::vector<hipEvent_t> events;
  minsr::GramJob* jobs = nullptr;   // device copy of the grouped Gram's job table
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void batch_release(minsr_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
  for (hipStream_t st : b->streams) (void)hipStreamDestroy(st);
  if (b->jobs) (void)hipFree(b->jobs);
  b->jobs = nullptr;
  b->exec = nullptr; b->graph = nullptr;
  b->events.clear(); b->streams.clear();
}

extern "C" {

int minsr_batch_create(minsr_model* const* models, const minsr_hamiltonian* hams,
                       const minsr_step_cfg* cfgs, const minsr_step_state* states,
                       const minsr_step_out* outs, int count, minsr_batch** out) {
  if (!models || !hams || !cfgs || !states || !outs || !out || count < 1)
    return fail(MINSR_E_INVALID_ARG, "null argument or empty batch");
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    if (!models[i]) return fail(MINSR_E_INVALID_ARG, "null model in batch");
    if (models[i]->linear)
      return fail(MINSR_E_UNSUPPORTED, "the linear test model has no minSR step");
    if (!states[i].dev_counter)
      return fail(MINSR_E_INVALID_ARG, "batch instances need a device-side Philox counter");
    for (int j = 0; j < i; ++j)
      if (models[j] == models[i]) return fail(MINSR_E_INVALID_ARG, "a model appears twice in a batch");
  }
  minsr_batch* b = new (std::nothrow) minsr_batch();
  if (!b) return fail(MINSR_E_NOMEM, "host allocation failed");
  b->models.assign(models, models + count);
  b->hams.assign(hams, hams + count);
  b->cfgs.assign(cfgs, cfgs + count);
  b->states.assign(states, states + count);
  b->outs.assign(outs, outs + count);
  // one stream per instance plus a library-owned origin stream for the
  // capture (the caller's stream may be the legacy null stream, which
  // cannot be captured; the instantiated graph is launched on it instead)
  for (int i = 0; i <= count; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      batch_release(b); delete b;
      return fail(MINSR_E_DEVICE, "stream creation failed");
    }
    b->streams.push_back(st);
  }
  for (int i = 0; i < 2 * (count + 1); ++i) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      batch_release(b); delete b;
      return fail(MINSR_E_DEVICE, "event creation failed");
    }
    b->events.push_back(e);
  }
  *out = b;
  return MINSR_OK;
}

// Phase-major capture: every instance's first stage on its own stream, then
// the Grams of the BF16 split-form instances in one grouped launch (each
// instance keeps the split its own step would use, so T is the same), then
// every instance's solve and update on its stream again.
static int batch_capture(minsr_batch* b) {
  const int count = (int)b->models.size();
  std::vector<minsr::GramJob> jobs;
  std::vector<int> grouped(count, 0);
  int items = 0, ritems = 0;
  for (int i = 0; i < count; ++i) {
    minsr_model* m = b->models[i];
    const minsr_step_cfg& c = b->cfgs[i];
    // an instance whose shape the step would reject runs the whole step
    // alone, which reports the error
    if (c.form != MINSR_FORM_BF16_FP64 || c.Ns < 2 || c.Ns > m->d.max_Ns) continue;
    const int n = (m->cplx ? 2 : 1) * c.Ns;
    const size_t Np = m->L.Np;
    const void* R = m->R;
    const void* Rlo = (const void*)((const __hip_bfloat16*)m->R + (size_t)n * padded_ld(Np));
    minsr::GramJob g{};
    int rc = gram_job(n, Np, R, Rlo, m->T, m->gpart, m->gpart_elems, m->tune_gram_split, &g);
    if (rc) return rc;
    g.item0 = items;
    g.ritem0 = ritems;
    items += g.npairs * g.S;
    ritems += g.npairs * minsr::GRAM_SUBTILES;
    jobs.push_back(g);
    grouped[i] = 1;
  }
  if (!jobs.empty()) {
    if (!b->jobs) MINSR_HIP(hipMalloc(&b->jobs, sizeof(minsr::GramJob) * count));
    MINSR_HIP(hipMemcpy(b->jobs, jobs.data(), sizeof(minsr::GramJob) * jobs.size(),
                        hipMemcpyHostToDevice));
  }
  hipStream_t s = b->streams.back();
  MINSR_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int rc = MINSR_OK;
  // stages of instance i on its stream, between a wait on `fork` and a
  // record of `join` that the origin stream waits for
  auto run = [&](int i, int stages, hipEvent_t fork, hipEvent_t join) {
    minsr_model* m = b->models[i];
    const int t_max = m->t_max;
    m->t_max = 0;   // no event timing inside the graph
    if (hipStreamWaitEvent(b->streams[i], fork, 0) != hipSuccess)
      rc = fail(MINSR_E_DEVICE, "fork wait failed");
    if (!rc) rc = step_stages(m, &b->hams[i], &b->cfgs[i], &b->states[i], &b->outs[i],
                              b->streams[i], stages);
    m->t_max = t_max;
    if (!rc && hipEventRecord(join, b->streams[i]) != hipSuccess)
      rc = fail(MINSR_E_DEVICE, "join record failed");
    if (!rc && hipStreamWaitEvent(s, join, 0) != hipSuccess)
      rc = fail(MINSR_E_DEVICE, "join wait failed");
  };
  if (hipEventRecord(b->events[0], s) != hipSuccess) rc = fail(MINSR_E_DEVICE, "fork record failed");
  for (int i = 0; i < count && !rc; ++i)
    run(i, grouped[i] ? 1 : 7, b->events[0], b->events[1 + i]);
  if (!rc && !jobs.empty()) {
    rc = launch_gram_grouped(b->jobs, (int)jobs.size(), items, ritems, s);
    if (!rc && hipEventRecord(b->events[count + 1], s) != hipSuccess)
      rc = fail(MINSR_E_DEVICE, "fork record failed");
    for (int i = 0; i < count && !rc; ++i)
      if (grouped[i]) run(i, 4, b->events[count + 1], b->events[count + 2 + i]);
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess || !g) return fail(MINSR_E_DEVICE, "graph capture failed");
  b->graph = g;
  MINSR_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return MINSR_OK;
}

int minsr_batch_step(minsr_batch* b, hipStream_t s) {
  if (!b) return fail(MINSR_E_INVALID_ARG, "null batch");
  if (!b->exec) {
    int rc = batch_capture(b);
    if (rc) return rc;
  }
  MINSR_HIP(hipGraphLaunch(b->exec, s));
  return MINSR_OK;
}

int minsr_batch_destroy(minsr_batch* b) {
  if (!b) return fail(MINSR_E_INVALID_ARG, "null batch");
  (void)hipDeviceSynchronize();
  batch_release(b);
  delete b;
  return MINSR_OK;
}
}  // extern "C"
