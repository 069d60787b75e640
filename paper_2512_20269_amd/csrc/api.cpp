// C ABI (include/iffd.h): argument validation, table upload and the host
// side of the PCG loop.  All arithmetic on vectors runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "dense2d.h"
#include "launch.h"
#include "pcg_state.h"
#include "plan.h"

namespace iffd {
hipError_t state_init(const Plan& P, char* st, int nslots, hipStream_t s);
hipError_t pcg_begin_dev(const Plan& P, char* st, int nslots, const int* h_slots, int count,
                         const double* f, double rtol, int maxit, hipStream_t s);
hipError_t pcg_iterate_dev(const Plan& P, char* st, int nslots, int k, hipStream_t s);
hipError_t pcg_take_dev(const Plan& P, char* st, int nslots, int slot, double* u, hipStream_t s);
hipError_t pcg_status_dev(const Plan& P, const char* st, int nslots, double* out, hipStream_t s);
}  // namespace iffd

using namespace iffd;


namespace {

thread_local std::string g_err;

// nslots each PCG state buffer was initialised with (iffd_pcg_state_init):
// every stepped call must name the same plan and slot count, since the
// offsets inside the buffer follow from them
struct StateRec {
  const iffd_plan* plan;
  int nslots;
};
std::mutex g_state_mu;
std::unordered_map<const void*, StateRec> g_states;

void state_register(const void* st, const iffd_plan* plan, int nslots) {
  std::lock_guard<std::mutex> lk(g_state_mu);
  g_states[st] = StateRec{plan, nslots};
}

bool state_matches(const void* st, const iffd_plan* plan, int nslots) {
  std::lock_guard<std::mutex> lk(g_state_mu);
  auto it = g_states.find(st);
  return it != g_states.end() && it->second.plan == plan && it->second.nslots == nslots;
}

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return IFFD_E_HIP;
}

bool aligned256(const void* p) { return ((uintptr_t)p & 255) == 0; }

// eigenvalues of a small symmetric tridiagonal matrix (diag a, off b) by
// cyclic Jacobi on the dense form; used for the CG-Lanczos estimate.
void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b, double& lmin,
                      double& lmax) {
  const int k = (int)a.size();
  std::vector<double> A((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) {
    A[(size_t)i * k + i] = a[i];
    if (i + 1 < k) A[(size_t)i * k + i + 1] = A[(size_t)(i + 1) * k + i] = b[i];
  }
  const double eps = 2.220446049250313e-16;
  for (int sweep = 0; sweep < 100; ++sweep) {
    bool rot = false;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        double apq = A[(size_t)p * k + q], app = A[(size_t)p * k + p], aqq = A[(size_t)q * k + q];
        if (std::fabs(apq) <= std::max(eps * std::sqrt(std::fabs(app * aqq)), 1e-300)) continue;
        rot = true;
        double th = (aqq - app) / (2 * apq);
        double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1));
        double c = 1 / std::sqrt(t * t + 1), s = t * c;
        for (int j = 0; j < k; ++j) {
          double x = A[(size_t)p * k + j], y = A[(size_t)q * k + j];
          A[(size_t)p * k + j] = c * x - s * y;
          A[(size_t)q * k + j] = s * x + c * y;
        }
        for (int j = 0; j < k; ++j) {
          double x = A[(size_t)j * k + p], y = A[(size_t)j * k + q];
          A[(size_t)j * k + p] = c * x - s * y;
          A[(size_t)j * k + q] = s * x + c * y;
        }
      }
    if (!rot) break;
  }
  lmin = 1e300;
  lmax = -1e300;
  for (int i = 0; i < k; ++i) {
    lmin = std::min(lmin, A[(size_t)i * k + i]);
    lmax = std::max(lmax, A[(size_t)i * k + i]);
  }
}

template <typename T>
void put(std::vector<char>& buf, size_t off, const std::vector<double>& v) {
  T* d = reinterpret_cast<T*>(buf.data() + off);
  for (size_t i = 0; i < v.size(); ++i) d[i] = (T)v[i];
}

}  // namespace

namespace iffd {
int set_last_error(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace iffd


namespace {

// outlier windows of one rotated outlier block (n_out x m): the entries decay
// geometrically away from the two ends; entries below 2^-30 (FP32 apply) or
// 2^-60 (FP64 apply) of the largest contribute below the working precision
// to the dots and the rank-n_out update, so only the two end windows are used
// Three windows for a direction with a repeated knot: the two ends and one
// around the knot (positions kc0 .. kc1 of the knot window): positions below
// the midpoint between the left end and the knot go to the left window, those
// above the midpoint between the knot and the right end to the right one, the
// rest to [kw0, kw1).  Overlapping windows fall back to every position.
void outlier_windows3(const std::vector<double>& Vt, int n_out, int m, int kc0, int kc1,
                      int* win32, int* win64, int* kwin32, int* kwin64) {
  const int a = kc0 / 2, b = (kc1 + m) / 2;
  for (int w = 0; w < 2; ++w) {
    int* win = w == 0 ? win32 : win64;
    int* kw = w == 0 ? kwin32 : kwin64;
    win[0] = m; win[1] = m; kw[0] = 0; kw[1] = 0;
    if (n_out == 0) continue;
    const double thr = std::ldexp(1.0, w == 0 ? -30 : -60);
    double mx = 0.0;
    for (double v : Vt) mx = std::max(mx, std::fabs(v));
    int lo = 0, hi = m, k0 = m, k1 = 0;
    for (int j = 0; j < m; ++j)
      for (int q = 0; q < n_out; ++q)
        if (std::fabs(Vt[(size_t)q * m + j]) > thr * mx) {
          if (j < a) lo = std::max(lo, j + 1);
          else if (j >= b) hi = std::min(hi, j);
          else { k0 = std::min(k0, j); k1 = std::max(k1, j + 1); }
        }
    if (k1 <= k0) { k0 = k1 = lo; }
    if (lo <= k0 && k1 <= hi && lo < hi) {
      win[0] = lo; win[1] = hi; kw[0] = k0; kw[1] = k1;
    }
  }
}

void outlier_windows(const std::vector<double>& Vt, int n_out, int m, int* win32, int* win64) {
  for (int w = 0; w < 2; ++w) {
    int* win = w == 0 ? win32 : win64;
    win[0] = m;
    win[1] = m;
    if (n_out == 0) continue;
    const double thr = std::ldexp(1.0, w == 0 ? -30 : -60);
    double mx = 0.0;
    for (double v : Vt) mx = std::max(mx, std::fabs(v));
    int lo = 0, hi = m;   // left window [0, lo), right window [hi, m)
    for (int j = 0; j < m; ++j)
      for (int q = 0; q < n_out; ++q)
        if (std::fabs(Vt[(size_t)q * m + j]) > thr * mx) {
          if (j < m / 2) lo = std::max(lo, j + 1);
          else hi = std::min(hi, j);
        }
    if (lo < hi) { win[0] = lo; win[1] = hi; }
  }
}

// table upload and outlier setup of a general plan: per direction one FP64
// and one FP32 blob (tw | tf | AL | AR | Vt | lam | s | Kb | Mb), the outlier
// pencil solved on the device straight into both blobs
// the element tables of a mapped domain's system matrix
hipError_t upload_geometry(const Plan& P, void* d_tables, hipStream_t s) {
  if (P.geo.kind == 0) return hipSuccess;
  return hipMemcpyAsync((char*)d_tables + P.geo.off, P.geo.tab.data(), 8 * P.geo.tab.size(),
                        hipMemcpyHostToDevice, s);
}

// Dense Qt = [V_reg U Dt^{-1}, V_out Q_out] of one direction in FP32, row i
// = dof i, column a = mode a (regular modes, then the Q_out-rotated outlier
// vectors), and its eigenvalues lam, for the small 2-D route; written once at
// setup with synchronous copies.
int put_dense_dir(char* b, size_t dq, size_t dl, int m, int n_reg, const std::vector<double>& Qreg,
                  const std::vector<double>& Vt, const std::vector<double>& lam) {
  std::vector<float> q((size_t)m * m), l(m);
  for (int i = 0; i < m; ++i)
    for (int a = 0; a < m; ++a)
      q[(size_t)i * m + a] = (float)(a < n_reg ? Qreg[(size_t)a * m + i] : Vt[(size_t)(a - n_reg) * m + i]);
  for (int a = 0; a < m; ++a) l[a] = (float)lam[a];
  hipError_t e = hipMemcpy(b + dq, q.data(), 4 * q.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b + dl, l.data(), 4 * l.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "dense Qt upload");
  return IFFD_OK;
}

int upload_dense2d(const Plan& P, char* b) {
  if (!P.gen) {
    if (P.Vt.size() != (size_t)P.n_out * P.m) return fail(IFFD_E_STATE, "outlier vectors missing");
    return put_dense_dir(b, P.lay.dq32, P.lay.dlam32, P.m, P.n_reg, P.Qreg, P.Vt, P.lam);
  }
  for (int k = 0; k < 2; ++k) {
    const GDir& G = P.dirs[k];
    if (G.Vt.size() != (size_t)G.n_out * G.m) return fail(IFFD_E_STATE, "outlier vectors missing");
    const int rc = put_dense_dir(b, G.dq32, G.dlam32, G.m, G.n_reg, G.Qreg, G.Vt, G.lam);
    if (rc != IFFD_OK) return rc;
  }
  return IFFD_OK;
}

int setup_general(Plan& P, void* d_tables, hipStream_t s) {
  std::vector<char> buf(P.lay.total, 0);
  for (int k = 0; k < P.d; ++k) {
    const GDir& G = P.dirs[k];
    std::vector<double> blob((size_t)G.len, 0.0);
    std::copy(G.tw.begin(), G.tw.end(), blob.begin() + G.o_tw);
    std::copy(G.tf.begin(), G.tf.end(), blob.begin() + G.o_tf);
    std::copy(G.AL.begin(), G.AL.end(), blob.begin() + G.o_al);
    std::copy(G.AR.begin(), G.AR.end(), blob.begin() + G.o_ar);
    std::copy(G.lam.begin(), G.lam.end(), blob.begin() + G.o_lam);
    std::copy(G.s.begin(), G.s.end(), blob.begin() + G.o_s);
    if (G.generic) {
      std::copy(G.LB.begin(), G.LB.begin() + (size_t)G.n_reg * G.bl, blob.begin() + G.o_lb);
      std::copy(G.UB.begin(), G.UB.end(), blob.begin() + G.o_ub);
    }
    std::copy(G.EW.begin(), G.EW.end(), blob.begin() + G.o_ew);
    // band rows padded from 2p+1 to 2pm+1 columns (centred)
    const int bw = 2 * G.p + 1, bwp = 2 * G.pm + 1, sh = G.pm - G.p;
    for (int i = 0; i < G.m; ++i)
      for (int o = 0; o < bw; ++o) {
        blob[(size_t)G.o_kb + (size_t)i * bwp + sh + o] = G.Kb[(size_t)i * bw + o];
        blob[(size_t)G.o_mb + (size_t)i * bwp + sh + o] = G.Mb[(size_t)i * bw + o];
      }
    put<double>(buf, G.blob64, blob);
    put<float>(buf, G.blob32, blob);
    if (P.method == IFFD_METHOD_DENSE_FD) {
      std::vector<double> QT((size_t)G.m * G.m);
      for (int i = 0; i < G.m; ++i)
        for (int j = 0; j < G.m; ++j) QT[(size_t)j * G.m + i] = G.Qfd[(size_t)i * G.m + j];
      put<double>(buf, G.fq64, G.Qfd);
      put<double>(buf, G.fqt64, QT);
      put<double>(buf, G.flam64, G.lamfd);
      put<float>(buf, G.fq32, G.Qfd);
      put<float>(buf, G.fqt32, QT);
      put<float>(buf, G.flam32, G.lamfd);
    }
    put<double>(buf, G.ao64, G.Ao);
    put<double>(buf, G.bo64, G.Bo);
    put<double>(buf, G.vout64, G.Vout);
  }
  {
    const int bwp = 2 * P.dirs[0].pm + 1;
    std::vector<double> unit((size_t)2 * bwp, 0.0);   // K = 0 | M = e_pm
    unit[(size_t)bwp + P.dirs[0].pm] = 1.0;
    put<double>(buf, P.lay.unit64, unit);
  }
  hipError_t e = hipMemcpyAsync(d_tables, buf.data(), buf.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = upload_geometry(P, d_tables, s);
  if (e != hipSuccess) return hip_fail(e, "table upload");
  char* b = (char*)d_tables;
  for (int k = 0; k < P.d && e == hipSuccess; ++k) {
    const GDir& G = P.dirs[k];
    e = launch_setup_outliers_at((const double*)(b + G.ao64), (const double*)(b + G.bo64),
                                 (const double*)(b + G.vout64), G.n_out, G.m, G.n_reg,
                                 (double*)(b + G.blob64) + G.o_lam, (float*)(b + G.blob32) + G.o_lam,
                                 (double*)(b + G.blob64) + G.o_vt, (float*)(b + G.blob32) + G.o_vt,
                                 (double*)(b + G.stat64), s);
  }
  if (e != hipSuccess) return hip_fail(e, "outlier setup");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "setup sync");
  for (int k = 0; k < P.d; ++k) {
    GDir& G = P.dirs[k];
    if (G.n_out == 0) {
      G.Vt.clear();
      outlier_windows(G.Vt, 0, G.m, G.win32, G.win64);
      continue;
    }
    std::vector<double> lam(G.m), vt((size_t)G.n_out * G.m);
    double stat = 0.0;
    e = hipMemcpy(&stat, b + G.stat64, 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
      e = hipMemcpy(lam.data(), b + G.blob64 + 8 * (size_t)G.o_lam, 8 * G.m, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
      e = hipMemcpy(vt.data(), b + G.blob64 + 8 * (size_t)G.o_vt, 8 * vt.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "setup readback");
    if (stat > 0.0)
      return fail(IFFD_E_INVAL, "direction " + std::to_string(k + 1) +
                                    ": outlier pencil mass block not positive definite at pivot " +
                                    std::to_string((int)stat));
    if (stat != 0.0)
      return fail(IFFD_E_INVAL, "direction " + std::to_string(k + 1) +
                                    ": outlier pencil eigenpairs not finite and positive");
    for (int j = G.n_reg; j < G.m; ++j) G.lam[j] = lam[j];
    G.Vt = vt;
    if (G.rk)
      outlier_windows3(G.Vt, G.n_out, G.m, G.wk0, G.wk1 + G.rk, G.win32, G.win64, G.kwin32, G.kwin64);
    else
      outlier_windows(G.Vt, G.n_out, G.m, G.win32, G.win64);
  }
  if (P.dense2d) return upload_dense2d(P, b);
  return IFFD_OK;
}

}  // namespace

extern "C" {

const char* iffd_last_error(void) { return g_err.c_str(); }

const char* iffd_status_string(int s) {
  switch (s) {
    case IFFD_OK: return "ok";
    case IFFD_W_NOT_CONVERGED: return "not converged";
    case IFFD_E_INVAL: return "invalid argument";
    case IFFD_E_UNSUPPORTED: return "unsupported";
    case IFFD_E_HIP: return "HIP error";
    case IFFD_E_BREAKDOWN: return "PCG breakdown";
    case IFFD_E_WORKSPACE: return "buffer too small";
    case IFFD_E_STATE: return "plan not ready";
    default: return "unknown status";
  }
}

int iffd_device_ok(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  return std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
}

int iffd_plan_create(iffd_plan** out, int d, int n, int p, const iffd_opts* opts) {
  if (!out) return fail(IFFD_E_INVAL, "out is null");
  *out = nullptr;
  iffd_plan* pl = new iffd_plan();
  std::string err;
  int rc = build_plan(pl->P, d, n, p, opts, err);
  if (rc != IFFD_OK) {
    delete pl;
    return fail(rc, err);
  }
  *out = pl;
  return IFFD_OK;
}

int iffd_plan_create_general(iffd_plan** out, int d, const int* n, const int* p,
                             const int* dirichlet, const iffd_opts* opts) {
  if (!out) return fail(IFFD_E_INVAL, "out is null");
  *out = nullptr;
  iffd_plan* pl = new iffd_plan();
  std::string err;
  int rc = build_plan_general(pl->P, d, n, p, dirichlet, opts, err);
  if (rc != IFFD_OK) {
    delete pl;
    return fail(rc, err);
  }
  *out = pl;
  return IFFD_OK;
}

int iffd_plan_query_dirs(const iffd_plan* plan, iffd_dir_info* h_out, int count) {
  if (!plan || !h_out) return fail(IFFD_E_INVAL, "null argument");
  const Plan& P = plan->P;
  if (count < P.d) return fail(IFFD_E_WORKSPACE, "fewer entries than directions");
  for (int k = 0; k < P.d; ++k) {
    iffd_dir_info& I = h_out[k];
    if (P.gen) {
      const GDir& G = P.dirs[k];
      I.n = G.n; I.p = G.p; I.dirichlet_lo = G.dlo; I.dirichlet_hi = G.dhi;
      const bool fft = P.method == IFFD_METHOD_FFT;
      I.m = G.m; I.n_reg = fft ? G.n_reg : G.m; I.n_out = fft ? G.n_out : 0;
      I.fft_len = fft ? G.L : 0;
    } else {
      const bool fft = P.method == IFFD_METHOD_FFT;
      I.n = P.n; I.p = P.p; I.dirichlet_lo = 1; I.dirichlet_hi = 1;
      I.m = P.m; I.n_reg = fft ? P.n_reg : P.m; I.n_out = fft ? P.n_out : 0;
      I.fft_len = fft ? P.L : 0;
    }
  }
  return IFFD_OK;
}

int iffd_plan_set_geometry(iffd_plan* plan, int kind, const double* h_params, int nparams) {
  if (!plan) return fail(IFFD_E_INVAL, "null argument");
  Plan& P = plan->P;
  if (P.ready) return fail(IFFD_E_STATE, "set the geometry before iffd_plan_setup");
  std::string err;
  const int rc = build_geometry(P, kind, h_params, nparams, err);
  if (rc != IFFD_OK) return fail(rc, err);
  return IFFD_OK;
}

int iffd_plan_set_knot(iffd_plan* plan, int direction, int k, int mult) {
  if (!plan) return fail(IFFD_E_INVAL, "null argument");
  Plan& P = plan->P;
  if (P.ready) return fail(IFFD_E_STATE, "set the knot before iffd_plan_setup");
  std::string err;
  const int rc = set_plan_knot(P, direction, k, mult, err);
  if (rc != IFFD_OK) return fail(rc, err);
  return IFFD_OK;
}

int iffd_plan_set_basis(iffd_plan* plan, int basis) {
  if (!plan) return fail(IFFD_E_INVAL, "null argument");
  Plan& P = plan->P;
  if (P.ready) return fail(IFFD_E_STATE, "set the basis before iffd_plan_setup");
  std::string err;
  const int rc = set_plan_basis(P, basis, err);
  if (rc != IFFD_OK) return fail(rc, err);
  return IFFD_OK;
}

void iffd_plan_destroy(iffd_plan* plan) {
  if (!plan) return;
  {
    std::lock_guard<std::mutex> lk(g_state_mu);
    for (auto it = g_states.begin(); it != g_states.end();)
      it = it->second.plan == plan ? g_states.erase(it) : std::next(it);
  }
  delete plan;
}

int iffd_plan_query(const iffd_plan* plan, iffd_plan_info* info) {
  if (!plan || !info) return fail(IFFD_E_INVAL, "null argument");
  const Plan& P = plan->P;
  info->d = P.d; info->n = P.n; info->p = P.p; info->m = P.m;
  info->n_reg = P.method == IFFD_METHOD_FFT ? P.n_reg : P.m;
  info->n_out = P.method == IFFD_METHOD_FFT ? P.n_out : 0;
  info->fft_len = P.method == IFFD_METHOD_FFT ? P.L : 0;
  info->method = P.method; info->apply_prec = P.prec; info->max_rhs = P.max_rhs;
  info->N = P.N;
  info->table_bytes = P.lay.total;
  info->apply_ws_bytes = apply_ws_bytes(P, P.max_rhs);
  info->pcg_ws_bytes = state_layout(P, P.max_rhs).total;
  info->matvec_ws_bytes = matvec_ws_bytes(P, P.max_rhs);
  const StateLayout one = state_layout(P, 1);
  info->state_bytes_per_slot = one.per_slot;
  info->state_bytes_fixed = one.fixed;
  return IFFD_OK;
}

int iffd_plan_setup(iffd_plan* plan, void* d_tables, size_t table_bytes, void* stream) {
  if (!plan || !d_tables) return fail(IFFD_E_INVAL, "null argument");
  Plan& P = plan->P;
  if (table_bytes < P.lay.total) return fail(IFFD_E_WORKSPACE, "table buffer too small");
  if (!aligned256(d_tables)) return fail(IFFD_E_INVAL, "table buffer must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  if (P.gen) {
    P.ready = false;
    const int rc = setup_general(P, d_tables, s);
    if (rc != IFFD_OK) return rc;
    P.d_tables = (char*)d_tables;
    P.table_bytes = table_bytes;
    P.ready = true;
    return IFFD_OK;
  }
  const TableLayout& t = P.lay;
  std::vector<char> buf(t.total, 0);
  put<double>(buf, t.lam64, P.lam);
  put<double>(buf, t.s64, P.s);
  put<double>(buf, t.v0_64, P.V0);
  put<double>(buf, t.v1_64, P.V1);
  put<double>(buf, t.twl64, P.twl);
  put<double>(buf, t.twp64, P.twp);
  put<double>(buf, t.kb64, P.Kb);
  put<double>(buf, t.mb64, P.Mb);
  put<double>(buf, t.kc64, P.Kc);
  put<double>(buf, t.mc64, P.Mc);
  put<double>(buf, t.ao64, P.Ao);
  put<double>(buf, t.bo64, P.Bo);
  put<double>(buf, t.vout64, P.Vout);
  put<float>(buf, t.lam32, P.lam);
  put<float>(buf, t.s32, P.s);
  put<float>(buf, t.v0_32, P.V0);
  put<float>(buf, t.v1_32, P.V1);
  put<float>(buf, t.twl32, P.twl);
  put<float>(buf, t.twp32, P.twp);
  if (P.method == IFFD_METHOD_DENSE_FD) {
    const int m = P.m;
    std::vector<double> QT((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) QT[(size_t)j * m + i] = P.Qfd[(size_t)i * m + j];
    put<double>(buf, t.qfd64, P.Qfd);
    put<double>(buf, t.qtfd64, QT);
    put<double>(buf, t.lamfd64, P.lamfd);
    put<float>(buf, t.qfd32, P.Qfd);
    put<float>(buf, t.qtfd32, QT);
    put<float>(buf, t.lamfd32, P.lamfd);
    if (P.prec == IFFD_PREC_F16S || P.prec == IFFD_PREC_BF16S) {
      // Q and Q^T in FP16 or BF16, scaled by the largest |entry| (in [-1, 1] after)
      double sq = 0.0;
      for (double v : P.Qfd) sq = std::max(sq, std::fabs(v));
      if (!(sq > 0.0)) sq = 1.0;
      if (P.prec == IFFD_PREC_F16S) {
        _Float16* q16 = (_Float16*)(buf.data() + t.qfd16);
        _Float16* qt16 = (_Float16*)(buf.data() + t.qtfd16);
        for (size_t k = 0; k < (size_t)m * m; ++k) {
          q16[k] = (_Float16)(P.Qfd[k] / sq);
          qt16[k] = (_Float16)(QT[k] / sq);
        }
      } else {
        __bf16* q16 = (__bf16*)(buf.data() + t.qfd16);
        __bf16* qt16 = (__bf16*)(buf.data() + t.qtfd16);
        for (size_t k = 0; k < (size_t)m * m; ++k) {
          q16[k] = (__bf16)(float)(P.Qfd[k] / sq);
          qt16[k] = (__bf16)(float)(QT[k] / sq);
        }
      }
      *(float*)(buf.data() + t.qs16) = (float)sq;
    }
  }
  hipError_t e = hipMemcpyAsync(d_tables, buf.data(), t.total, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = upload_geometry(P, d_tables, s);
  if (e != hipSuccess) return hip_fail(e, "table upload");
  P.d_tables = (char*)d_tables;
  P.table_bytes = table_bytes;
  if (P.method == IFFD_METHOD_FFT) {
    e = launch_setup_outliers(P, s);
    if (e != hipSuccess) return hip_fail(e, "outlier setup");
  }
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "setup sync");
  if (P.method == IFFD_METHOD_FFT && P.n_out > 0) {
    std::vector<double> lam(P.m), vt((size_t)P.n_out * P.m);
    double stat = 0.0;
    e = hipMemcpy(&stat, (char*)d_tables + t.stat64, 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
      e = hipMemcpy(lam.data(), (char*)d_tables + t.lam64, 8 * P.m, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
      e = hipMemcpy(vt.data(), (char*)d_tables + t.vt64, 8 * vt.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "setup readback");
    if (stat > 0.0)
      return fail(IFFD_E_INVAL, "outlier pencil: mass block not positive definite at pivot " +
                                    std::to_string((int)stat));
    if (stat != 0.0) return fail(IFFD_E_INVAL, "outlier pencil: non-finite or non-positive eigenpairs");
    for (int k = P.n_reg; k < P.m; ++k) P.lam[k] = lam[k];
    P.Vt = vt;
  }
  outlier_windows(P.Vt, P.method == IFFD_METHOD_FFT ? P.n_out : 0, P.m, P.win32, P.win64);
  if (P.method == IFFD_METHOD_FFT) {
    // the line-pass tables as one contiguous blob (one load sweep per block)
    std::vector<double> blob((size_t)P.blob_len, 0.0);
    std::copy(P.twl.begin(), P.twl.end(), blob.begin() + P.bo_twl);
    std::copy(P.twp.begin(), P.twp.end(), blob.begin() + P.bo_twp);
    std::copy(P.sn.begin(), P.sn.end(), blob.begin() + P.bo_sn);
    std::copy(P.Vt.begin(), P.Vt.end(), blob.begin() + P.bo_vt);
    std::copy(P.V0.begin(), P.V0.end(), blob.begin() + P.bo_v0);
    std::copy(P.V1.begin(), P.V1.end(), blob.begin() + P.bo_v1);
    std::copy(P.lam.begin(), P.lam.end(), blob.begin() + P.bo_lam);
    std::copy(P.s.begin(), P.s.end(), blob.begin() + P.bo_s);
    std::vector<char> bb(12 * blob.size() + 16, 0);
    std::memcpy(bb.data(), blob.data(), 8 * blob.size());
    for (size_t i = 0; i < blob.size(); ++i) {
      const float f = (float)blob[i];
      std::memcpy(bb.data() + 8 * blob.size() + 4 * i, &f, 4);
    }
    e = hipMemcpy((char*)d_tables + t.blob64, bb.data(), 8 * blob.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy((char*)d_tables + t.blob32, bb.data() + 8 * blob.size(), 4 * blob.size(),
                    hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "blob upload");
  }
  if (P.dense2d) {
    const int rc = upload_dense2d(P, (char*)d_tables);
    if (rc != IFFD_OK) return rc;
  }
  P.ready = true;
  return IFFD_OK;
}

int iffd_plan_read_dir(const iffd_plan* plan, int direction, int what, double* h_out,
                       size_t count, void* stream) {
  if (!plan || !h_out) return fail(IFFD_E_INVAL, "null argument");
  const Plan& P = plan->P;
  if (direction < 1 || direction > P.d) return fail(IFFD_E_INVAL, "direction out of range");
  if (!P.gen) return iffd_plan_read(plan, what, h_out, count, stream);
  const GDir& G = P.dirs[direction - 1];
  const std::vector<double>* v = nullptr;
  switch (what) {
    case 0: v = P.method == IFFD_METHOD_DENSE_FD ? &G.lamfd : &G.lam; break;
    case 1: v = &G.Dt; break;
    case 2: case 7: v = &G.Kb; break;
    case 3: v = &G.Mb; break;
    case 4: v = &G.AL; break;
    case 5: v = &G.AR; break;
    case 6:
      if (!P.ready) return fail(IFFD_E_STATE, "Vt is available after iffd_plan_setup");
      v = &G.Vt;
      break;
    default: return fail(IFFD_E_INVAL, "unknown table id");
  }
  if (count < v->size()) return fail(IFFD_E_WORKSPACE, "output array too small");
  std::copy(v->begin(), v->end(), h_out);
  return IFFD_OK;
}

int iffd_plan_read(const iffd_plan* plan, int what, double* h_out, size_t count, void* stream) {
  if (!plan || !h_out) return fail(IFFD_E_INVAL, "null argument");
  const Plan& P = plan->P;
  if (P.gen) return iffd_plan_read_dir(plan, 1, what, h_out, count, stream);
  const std::vector<double>* v = nullptr;
  switch (what) {
    case 0: v = &P.lam; break;
    case 1: v = &P.Dt; break;
    case 2: v = &P.Kb; break;
    case 3: v = &P.Mb; break;
    case 4: v = &P.V0; break;
    case 5: v = &P.V1; break;
    case 6:
      if (!P.ready) return fail(IFFD_E_STATE, "Vt is available after iffd_plan_setup");
      v = &P.Vt;
      break;
    case 7: v = &P.Kop; break;
    default: return fail(IFFD_E_INVAL, "unknown table id");
  }
  if (count < v->size()) return fail(IFFD_E_WORKSPACE, "output array too small");
  std::copy(v->begin(), v->end(), h_out);
  return IFFD_OK;
}

int iffd_precond_apply(const iffd_plan* plan, const double* d_r, double* d_z, int nrhs, void* d_ws,
                       size_t ws_bytes, void* stream) {
  if (!plan || !d_r || !d_z) return fail(IFFD_E_INVAL, "null argument");
  const Plan& P = plan->P;
  if (!P.ready) return fail(IFFD_E_STATE, "plan not set up");
  if (nrhs < 1 || nrhs > P.max_rhs) return fail(IFFD_E_INVAL, "nrhs out of range");
  if ((const void*)d_r == (const void*)d_z) return fail(IFFD_E_INVAL, "r and z must not alias");
  const size_t need = apply_ws_bytes(P, nrhs);
  if (need && (!d_ws || ws_bytes < need)) return fail(IFFD_E_WORKSPACE, "apply workspace too small");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = (P.method == IFFD_METHOD_FFT)
                     ? launch_iffd_apply(P, d_r, d_z, nrhs, d_ws, nullptr, 0, s)
                     : launch_fd_apply(P, d_r, d_z, nrhs, d_ws, nullptr, 0, s);
  if (e != hipSuccess) return hip_fail(e, "precond_apply launch");
  return IFFD_OK;
}

int iffd_apply_pass_count(const iffd_plan* plan) {
  if (!plan) return fail(IFFD_E_INVAL, "null argument");
  return plan->P.method == IFFD_METHOD_FFT ? 2 * plan->P.d - 1 : 0;
}

int iffd_apply_pass(const iffd_plan* plan, int pass, const double* d_r, double* d_z, int nrhs,
                    void* d_ws, size_t ws_bytes, void* stream) {
  if (!plan || !d_r || !d_z) return fail(IFFD_E_INVAL, "null argument");
  const Plan& P = plan->P;
  if (!P.ready) return fail(IFFD_E_STATE, "plan not set up");
  if (P.method != IFFD_METHOD_FFT) return fail(IFFD_E_STATE, "passes exist for the FFT method only");
  if (pass < 0 || pass >= 2 * P.d - 1) return fail(IFFD_E_INVAL, "pass out of range");
  if (nrhs < 1 || nrhs > P.max_rhs) return fail(IFFD_E_INVAL, "nrhs out of range");
  if ((const void*)d_r == (const void*)d_z) return fail(IFFD_E_INVAL, "r and z must not alias");
  const size_t need = apply_ws_bytes(P, nrhs);
  if (need && (!d_ws || ws_bytes < need)) return fail(IFFD_E_WORKSPACE, "apply workspace too small");
  hipError_t e = launch_iffd_pass(P, pass, d_r, d_z, nrhs, d_ws, nullptr, 0, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "apply pass launch");
  return IFFD_OK;
}

int iffd_plan_set_variant(iffd_plan* plan, int pass, int variant) {
  if (!plan) return fail(IFFD_E_INVAL, "null argument");
  if (plan->P.gen) return fail(IFFD_E_UNSUPPORTED, "general plans have a single FFT shape");
  if (pass < 0 || pass >= 2 * plan->P.d - 1 || variant < 0 || variant > 4)
    return fail(IFFD_E_INVAL, "pass or variant out of range");
  plan->P.variant[pass] = variant;
  return IFFD_OK;
}

int iffd_plan_get_variant(const iffd_plan* plan, int pass) {
  if (!plan) return fail(IFFD_E_INVAL, "null argument");
  if (pass < 0 || pass >= 2 * plan->P.d - 1) return fail(IFFD_E_INVAL, "pass out of range");
  if (plan->P.gen) return 1;
  return plan->P.variant[pass];
}

int iffd_plan_set_route(iffd_plan* plan, int route) {
  if (!plan) return fail(IFFD_E_INVAL, "null argument");
  if (route != IFFD_ROUTE_AUTO && route != IFFD_ROUTE_PASSES && route != IFFD_ROUTE_DENSE2D)
    return fail(IFFD_E_INVAL, "unknown route");
  if (route == IFFD_ROUTE_DENSE2D && !plan->P.dense2d)
    return fail(IFFD_E_UNSUPPORTED,
                "the dense 2-D route needs d = 2, the FFT method, an FP32 apply with p <= 4 and m <= 128");
  plan->P.route = route;
  return IFFD_OK;
}

int iffd_plan_get_route(const iffd_plan* plan, int nrhs) {
  if (!plan) return fail(IFFD_E_INVAL, "null argument");
  if (nrhs < 1) return fail(IFFD_E_INVAL, "nrhs out of range");
  if (plan->P.method != IFFD_METHOD_FFT) return IFFD_ROUTE_PASSES;
  return dense2d_route(plan->P, nrhs);
}

int iffd_plan_tune(iffd_plan* plan, void* d_scratch, size_t scratch_bytes, int reps, void* stream) {
  if (!plan || !d_scratch) return fail(IFFD_E_INVAL, "null argument");
  Plan& P = plan->P;
  if (!P.ready) return fail(IFFD_E_STATE, "plan not set up");
  if (P.method != IFFD_METHOD_FFT || P.gen) return IFFD_OK;
  const size_t need = 16 * (size_t)P.N + apply_ws_bytes(P, 1);
  if (scratch_bytes < need) return fail(IFFD_E_WORKSPACE, "tuning scratch too small");
  if (!aligned256(d_scratch)) return fail(IFFD_E_INVAL, "scratch must be 256-byte aligned");
  if (reps < 1) reps = 1;
  hipStream_t s = (hipStream_t)stream;
  double* r = (double*)d_scratch;
  double* z = r + P.N;
  void* ws = (char*)d_scratch + 16 * (size_t)P.N;
  hipError_t e = hipMemsetAsync(d_scratch, 0, need, s);
  if (e != hipSuccess) return hip_fail(e, "tune memset");
  hipEvent_t a, b;
  if ((e = hipEventCreate(&a)) != hipSuccess) return hip_fail(e, "tune event");
  if ((e = hipEventCreate(&b)) != hipSuccess) { hipEventDestroy(a); return hip_fail(e, "tune event"); }
  int rc = IFFD_OK;
  for (int k = 0; k < 2 * P.d - 1 && rc == IFFD_OK; ++k) {
    float best = 1e30f;
    int best_v = P.variant[k];
    // variants 3 and 4 exist for power-of-two transform lengths up to 256 only
    const int nvar = ((P.L & (P.L - 1)) == 0 && P.L <= 256) ? 5 : 3;
    for (int v = 0; v < nvar && rc == IFFD_OK; ++v) {
      P.variant[k] = v;
      for (int w = 0; w < 2; ++w) launch_iffd_pass(P, k, r, z, 1, ws, nullptr, 0, s);
      hipEventRecord(a, s);
      for (int i = 0; i < reps; ++i) e = launch_iffd_pass(P, k, r, z, 1, ws, nullptr, 0, s);
      hipEventRecord(b, s);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      if (e != hipSuccess) { rc = hip_fail(e, "tune launch"); break; }
      if (ms < best) { best = ms; best_v = v; }
    }
    P.variant[k] = best_v;
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  return rc;
}

int iffd_kron_matvec(const iffd_plan* plan, const double* d_x, double* d_y, int nrhs, void* d_ws,
                     size_t ws_bytes, void* stream) {
  if (!plan || !d_x || !d_y) return fail(IFFD_E_INVAL, "null argument");
  const Plan& P = plan->P;
  if (!P.ready) return fail(IFFD_E_STATE, "plan not set up");
  if (nrhs < 1 || nrhs > P.max_rhs) return fail(IFFD_E_INVAL, "nrhs out of range");
  if ((const void*)d_x == (const void*)d_y) return fail(IFFD_E_INVAL, "x and y must not alias");
  const size_t need = matvec_ws_bytes(P, nrhs);
  if (need && (!d_ws || ws_bytes < need)) return fail(IFFD_E_WORKSPACE, "matvec workspace too small");
  hipError_t e = launch_matvec(P, d_x, d_y, nrhs, d_ws, nullptr, 0, nullptr, 0, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "kron_matvec launch");
  return IFFD_OK;
}

// ---- stepped PCG -------------------------------------------------------------

int iffd_pcg_state_init(const iffd_plan* plan, void* d_state, size_t state_bytes, int nslots,
                        void* stream) {
  if (!plan || !d_state) return fail(IFFD_E_INVAL, "null argument");
  const Plan& P = plan->P;
  if (!P.ready) return fail(IFFD_E_STATE, "plan not set up");
  if (nslots < 1 || nslots > P.max_rhs) return fail(IFFD_E_INVAL, "nslots must be in 1..max_rhs");
  if (!aligned256(d_state)) return fail(IFFD_E_INVAL, "state must be 256-byte aligned");
  if (state_bytes < state_layout(P, nslots).total) return fail(IFFD_E_WORKSPACE, "state buffer too small");
  hipError_t e = state_init(P, (char*)d_state, nslots, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "state init");
  state_register(d_state, plan, nslots);
  return IFFD_OK;
}

int iffd_pcg_begin(const iffd_plan* plan, void* d_state, int nslots, const int* h_slots, int count,
                   const double* d_f, double rtol, int maxit, void* stream) {
  if (!plan || !d_state || !h_slots || !d_f) return fail(IFFD_E_INVAL, "null argument");
  const Plan& P = plan->P;
  if (!P.ready) return fail(IFFD_E_STATE, "plan not set up");
  if (!state_matches(d_state, plan, nslots))
    return fail(IFFD_E_STATE, "state not initialised for this plan with this nslots");
  if (count < 1 || count > nslots) return fail(IFFD_E_INVAL, "bad slot count");
  if (!(rtol >= 0.0) || maxit < 0) return fail(IFFD_E_INVAL, "bad rtol / maxit");
  std::vector<char> seen(nslots, 0);
  for (int k = 0; k < count; ++k) {
    if (h_slots[k] < 0 || h_slots[k] >= nslots || seen[h_slots[k]])
      return fail(IFFD_E_INVAL, "slot indices must be distinct and < nslots");
    seen[h_slots[k]] = 1;
  }
  if (P.method == IFFD_METHOD_FFT || P.method == IFFD_METHOD_DENSE_FD) {
    if (nslots > P.max_rhs) return fail(IFFD_E_INVAL, "nslots exceeds the plan's max_rhs");
  }
  hipError_t e = pcg_begin_dev(P, (char*)d_state, nslots, h_slots, count, d_f, rtol, maxit,
                               (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "pcg begin");
  return IFFD_OK;
}

int iffd_pcg_iterate(const iffd_plan* plan, void* d_state, int nslots, int k, void* stream) {
  if (!plan || !d_state) return fail(IFFD_E_INVAL, "null argument");
  const Plan& P = plan->P;
  if (!P.ready) return fail(IFFD_E_STATE, "plan not set up");
  if (nslots < 1 || nslots > P.max_rhs || k < 0) return fail(IFFD_E_INVAL, "bad nslots / k");
  if (!state_matches(d_state, plan, nslots))
    return fail(IFFD_E_STATE, "state not initialised for this plan with this nslots");
  hipError_t e = pcg_iterate_dev(P, (char*)d_state, nslots, k, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "pcg iterate");
  return IFFD_OK;
}

int iffd_pcg_poll(const iffd_plan* plan, const void* d_state, int nslots, double* h_out,
                  void* stream) {
  if (!plan || !d_state || !h_out) return fail(IFFD_E_INVAL, "null argument");
  const Plan& P = plan->P;
  if (nslots < 1 || nslots > P.max_rhs) return fail(IFFD_E_INVAL, "nslots must be in 1..max_rhs");
  if (!state_matches(d_state, plan, nslots))
    return fail(IFFD_E_STATE, "state not initialised for this plan with this nslots");
  const StateLayout L = state_layout(P, nslots);
  std::vector<double> sc((size_t)nslots * kScal);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(sc.data(), (const char*)d_state + L.scal, 8 * sc.size(),
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "pcg poll");
  for (int i = 0; i < nslots; ++i) {
    const double* r = &sc[(size_t)i * kScal];
    h_out[4 * i + 0] = r[S_ACTIVE];
    h_out[4 * i + 1] = r[S_USED] != 0.0 ? r[S_STATUS] : -100.0;
    h_out[4 * i + 2] = r[S_IT];
    h_out[4 * i + 3] = r[S_RELRES];
  }
  return IFFD_OK;
}

int iffd_pcg_status(const iffd_plan* plan, const void* d_state, int nslots, double* d_out,
                    void* stream) {
  if (!plan || !d_state || !d_out) return fail(IFFD_E_INVAL, "null argument");
  if (nslots < 1 || nslots > plan->P.max_rhs) return fail(IFFD_E_INVAL, "nslots must be in 1..max_rhs");
  if (!plan->P.ready) return fail(IFFD_E_STATE, "plan not set up");
  if (!state_matches(d_state, plan, nslots))
    return fail(IFFD_E_STATE, "state not initialised for this plan with this nslots");
  hipError_t e = pcg_status_dev(plan->P, (const char*)d_state, nslots, d_out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "pcg status");
  return IFFD_OK;
}

int iffd_pcg_take(const iffd_plan* plan, void* d_state, int nslots, int slot, double* d_u,
                  void* stream) {
  if (!plan || !d_state || !d_u) return fail(IFFD_E_INVAL, "null argument");
  if (nslots < 1 || nslots > plan->P.max_rhs) return fail(IFFD_E_INVAL, "nslots must be in 1..max_rhs");
  if (slot < -1 || slot >= nslots) return fail(IFFD_E_INVAL, "slot out of range");
  if (!plan->P.ready) return fail(IFFD_E_STATE, "plan not set up");
  if (!state_matches(d_state, plan, nslots))
    return fail(IFFD_E_STATE, "state not initialised for this plan with this nslots");
  hipError_t e = pcg_take_dev(plan->P, (char*)d_state, nslots, slot, d_u, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "pcg take");
  return IFFD_OK;
}

int iffd_pcg_solve(const iffd_plan* plan, const double* d_f, double* d_u, int nrhs, double rtol,
                   int maxit, int check_every, iffd_pcg_stats* h_stats, void* d_ws,
                   size_t ws_bytes, void* stream) {
  if (!plan || !d_f || !d_u || !d_ws) return fail(IFFD_E_INVAL, "null argument");
  const Plan& P = plan->P;
  if (!P.ready) return fail(IFFD_E_STATE, "plan not set up");
  if (nrhs < 1 || nrhs > P.max_rhs) return fail(IFFD_E_INVAL, "nrhs out of range");
  if (!(rtol >= 0.0) || maxit < 0) return fail(IFFD_E_INVAL, "bad rtol / maxit");
  const StateLayout L = state_layout(P, nrhs);
  if (ws_bytes < L.total) return fail(IFFD_E_WORKSPACE, "pcg workspace too small");
  if (!aligned256(d_ws)) return fail(IFFD_E_INVAL, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  char* st = (char*)d_ws;
  int rc = iffd_pcg_state_init(plan, d_ws, ws_bytes, nrhs, stream);
  if (rc != IFFD_OK) return rc;
  std::vector<int> slots(nrhs);
  for (int k = 0; k < nrhs; ++k) slots[k] = k;
  rc = iffd_pcg_begin(plan, d_ws, nrhs, slots.data(), nrhs, d_f, rtol, maxit, stream);
  if (rc != IFFD_OK) return rc;
  // Pipelined polling: the next batch of iterations is enqueued before the
  // host waits for the previous batch's slot records (copied to pinned host
  // memory), so the device never idles on the host.  Converged slots make the
  // extra batch a no-op.
  const int step = check_every > 0 ? check_every : 1;
  const size_t rec = (size_t)4 * nrhs;
  static thread_local double* hbuf = nullptr;
  static thread_local size_t hcap = 0;
  if (hcap < 2 * rec) {
    if (hbuf) (void)hipHostFree(hbuf);
    hbuf = nullptr;
    hcap = 0;
    hipError_t e = hipHostMalloc((void**)&hbuf, 2 * rec * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "pinned status buffer");
    hcap = 2 * rec;
  }
  double* dstat = (double*)(st + L.stat);
  hipEvent_t ev[2] = {nullptr, nullptr};
  for (int i = 0; i < 2; ++i) {
    hipError_t e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "event");
  }
  auto post_status = [&](int b) -> hipError_t {
    hipError_t e = pcg_status_dev(P, st, nrhs, dstat + b * rec, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hbuf + b * rec, dstat + b * rec, rec * sizeof(double),
                         hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(ev[b], s);
    return e;
  };
  hipError_t pe = post_status(0);   // the slots right after begin
  int done_it = 0, cur = 0;
  while (pe == hipSuccess) {
    const int kk = std::min(step, maxit - done_it);
    if (kk > 0) {
      pe = pcg_iterate_dev(P, st, nrhs, kk, s);
      if (pe == hipSuccess) pe = post_status(cur ^ 1);
      if (pe != hipSuccess) break;
      done_it += kk;
    }
    pe = hipEventSynchronize(ev[cur]);
    if (pe != hipSuccess) break;
    bool any = false;
    for (int k = 0; k < nrhs; ++k) any = any || hbuf[cur * rec + 4 * k] != 0.0;
    if (!any || kk == 0) break;
    cur ^= 1;
  }
  for (int i = 0; i < 2; ++i) (void)hipEventDestroy(ev[i]);
  if (pe != hipSuccess) return hip_fail(pe, "pcg iterate");
  // solution out, true residual
  double* x = (double*)(st + L.x);
  double* qz = (double*)(st + L.qz);
  double* part = (double*)(st + L.part);
  hipError_t e = hipMemcpyAsync(d_u, x, 8 * (size_t)P.N * nrhs, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "copy solution");
  // true residual: ||f - A u||^2 partials straight from the operator
  e = launch_matvec(P, d_u, qz, nrhs, L.mvws ? st + L.mvws : nullptr, part, L.npart, nullptr, 0,
                    s, d_f);
  if (e != hipSuccess) return hip_fail(e, "true residual");
  const int nb = matvec_blocks(P), stride = L.npart;
  std::vector<double> parts((size_t)nrhs * stride), sc((size_t)nrhs * kScal),
      hist((size_t)nrhs * kHist * 2);
  e = hipMemcpyAsync(parts.data(), part, 8 * parts.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sc.data(), st + L.scal, 8 * sc.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hist.data(), st + L.hist, 8 * hist.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "stats readback");
  int worst = IFFD_OK;
  for (int k = 0; k < nrhs; ++k) {
    const double* rec = &sc[(size_t)k * kScal];
    double rr = 0.0;
    for (int i = 0; i < nb; ++i) rr += parts[(size_t)k * stride + i];
    const int status = (int)rec[S_STATUS];
    if (status < 0) worst = std::min(worst, status);
    else if (worst >= 0) worst = std::max(worst, status);
    if (h_stats) {
      iffd_pcg_stats& S = h_stats[k];
      S.iterations = (int)rec[S_IT];
      S.converged = rec[S_CONV] != 0.0;
      S.status = status;
      S.relres = rec[S_RELRES];
      S.relres_true = rec[S_FF] > 0 ? std::sqrt(rr / rec[S_FF]) : 0.0;
      // CG-Lanczos: T_jj = 1/a_j + b_{j-1}/a_{j-1}, T_j,j+1 = sqrt(b_j)/a_j
      const int kl = std::min(S.iterations, kHist);
      S.lanczos_lmin = S.lanczos_lmax = S.kappa_est = 0.0;
      if (kl >= 1) {
        const double* h = &hist[(size_t)k * kHist * 2];
        std::vector<double> a(kl), b(kl > 1 ? kl - 1 : 0);
        for (int j = 0; j < kl; ++j) {
          a[j] = 1.0 / h[2 * j];
          if (j > 0) a[j] += h[2 * (j - 1) + 1] / h[2 * (j - 1)];
          if (j + 1 < kl) b[j] = std::sqrt(h[2 * j + 1]) / h[2 * j];
        }
        double lmin, lmax;
        tridiag_extremes(a, b, lmin, lmax);
        S.lanczos_lmin = lmin;
        S.lanczos_lmax = lmax;
        S.kappa_est = lmin > 0 ? lmax / lmin : 0.0;
      }
    }
  }
  return worst;
}

}  // extern "C"
