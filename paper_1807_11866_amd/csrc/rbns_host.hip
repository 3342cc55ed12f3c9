// rbns_host.hip -- host side of the C ABI declared in include/rbns.h: contexts, HBM budget,
// resident tensor sets, packed operands, per-stream workspaces and kernel launches.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/rbns.h"
#include "rb_kernels.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(RB_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));            \
  } while (0)

inline int64_t ceil_to(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Pack {              // packed MFMA operand for one basis size
  DevBuf buf;
  int nrb = 0, nks_s = 0, nks = 0;
};

struct Set {
  int N = 0, Q = 0, Qc = 0, Qf = 0, Np = 0, Qb = 0;
  DevBuf A, C, F, H, BpT, Asv, Csv, Fs;
  bool hasH = false;
  std::map<int, Pack> solve_f64;                     // key: N
  std::map<std::pair<int, int>, Pack> press_f64;     // key: (N, Np)
};

struct Workspace {
  DevBuf buf;            // Newton state of the last batch on this stream (see NewtonState)
};

}  // namespace

struct TimedLaunch {
  int family;
  hipEvent_t start, stop;
};

struct rb_ctx {
  int device = 0;
  size_t budget = 0, used = 0;
  std::vector<std::unique_ptr<Set>> sets;
  std::map<void*, Workspace> ws;
  std::mutex mu;
  bool timing = false;
  std::vector<TimedLaunch> timed;       // recorded, not yet read
  std::vector<hipEvent_t> event_pool;
};

namespace {

int dev_alloc(rb_ctx* c, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (c->budget && c->used + bytes > c->budget)
    return fail(RB_E_NOMEM, "HBM budget exceeded: need %zu more bytes, %zu of %zu in use",
                bytes, c->used, c->budget);
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail(RB_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  b.bytes = bytes;
  c->used += bytes;
  return RB_OK;
}

void dev_free(rb_ctx* c, DevBuf& b) {
  if (b.p) {
    (void)hipFree(b.p);
    c->used -= b.bytes;
  }
  b.p = nullptr;
  b.bytes = 0;
}

int upload(rb_ctx* c, DevBuf& b, const double* host, size_t n) {
  int rc = dev_alloc(c, b, n * sizeof(double));
  if (rc) return rc;
  HIP_TRY(hipMemcpy(b.p, host, n * sizeof(double), hipMemcpyHostToDevice));
  return RB_OK;
}

int use_device(rb_ctx* c) {
  HIP_TRY(hipSetDevice(c->device));
  return RB_OK;
}

Set* get_set(rb_ctx* c, int id) {
  if (id < 0 || id >= (int)c->sets.size() || !c->sets[id]) return nullptr;
  return c->sets[id].get();
}

int launch_grid(int64_t total) {
  int64_t g = (total + 255) / 256;
  return (int)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

// Solve operand for basis size N (built once on the device, then cached).
int solve_pack_f64(rb_ctx* c, Set* s, int N, Pack** out) {
  auto it = s->solve_f64.find(N);
  if (it != s->solve_f64.end()) { *out = &it->second; return RB_OK; }
  Pack p;
  p.nrb = (int)(ceil_to((int64_t)N * N, 16) / 16);
  p.nks_s = (int)(ceil_to((int64_t)s->Qc * N, 4) / 4);
  p.nks = p.nks_s + (int)(ceil_to(s->Q, 4) / 4);
  const int64_t total = (int64_t)p.nrb * p.nks * 64;
  int rc = dev_alloc(c, p.buf, total * sizeof(double));
  if (rc) return rc;
  hipLaunchKernelGGL(rb::pack_solve_f64, dim3(launch_grid(total)), dim3(256), 0, 0,
                     (const double*)s->C.p, (const double*)s->A.p, s->N, N, s->Q, s->Qc,
                     p.nrb, p.nks, p.nks_s, (double*)p.buf.p);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipDeviceSynchronize());
  auto ins = s->solve_f64.emplace(N, p);
  *out = &ins.first->second;
  return RB_OK;
}

int press_pack_f64(rb_ctx* c, Set* s, int N, int Np, Pack** out) {
  auto key = std::make_pair(N, Np);
  auto it = s->press_f64.find(key);
  if (it != s->press_f64.end()) { *out = &it->second; return RB_OK; }
  Pack p;
  p.nrb = (int)(ceil_to((int64_t)N * Np, 16) / 16);
  p.nks_s = (int)(ceil_to((int64_t)s->Qc * N, 4) / 4);
  p.nks = p.nks_s + (int)(ceil_to(s->Q, 4) / 4);
  const int64_t total = (int64_t)p.nrb * p.nks * 64;
  int rc = dev_alloc(c, p.buf, total * sizeof(double));
  if (rc) return rc;
  hipLaunchKernelGGL(rb::pack_pressure_f64, dim3(launch_grid(total)), dim3(256), 0, 0,
                     (const double*)s->Csv.p, (const double*)s->Asv.p, s->N, s->Np, N, Np,
                     s->Q, s->Qc, p.nrb, p.nks, p.nks_s, (double*)p.buf.p);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipDeviceSynchronize());
  auto ins = s->press_f64.emplace(key, p);
  *out = &ins.first->second;
  return RB_OK;
}

int workspace(rb_ctx* c, void* stream, size_t bytes, Workspace** out) {
  Workspace& w = c->ws[stream];
  if (w.buf.bytes < bytes) {
    if (w.buf.p) {
      // the previous buffer may still be in use by work queued on this stream
      HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
      dev_free(c, w.buf);
    }
    int rc = dev_alloc(c, w.buf, bytes);
    if (rc) return rc;
  }
  *out = &w;
  return RB_OK;
}

// Carve the Newton state for Bp (padded) requests out of one workspace allocation.
size_t newton_state_bytes(int64_t Bp, int NP, int64_t mp) {
  return (size_t)(Bp * mp + 3 * Bp * NP) * sizeof(double) + (size_t)3 * Bp * sizeof(int) + 256;
}

rb::NewtonState carve_state(void* base, int64_t Bp, int NP, int64_t mp) {
  rb::NewtonState s;
  double* d = (double*)base;
  s.J = d;
  d += Bp * mp;
  s.U = d;
  d += Bp * NP;
  s.Fv = d;
  d += Bp * NP;
  s.Wv = d;
  d += Bp * NP;
  int* ip = (int*)d;
  s.done = ip;
  s.iters = ip + Bp;
  s.status = ip + 2 * Bp;
  s.mp = mp;
  s.NP = NP;
  return s;
}

int np_bucket(int n) { return (int)ceil_to(n, 8); }

enum { FAM_JACOBIAN = 0, FAM_LU = 1, FAM_PRESSURE = 2, FAM_COUNT = 3 };
const char* const kFamilies[FAM_COUNT] = {"jacobian", "lu", "pressure"};

hipEvent_t take_event(rb_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one kernel launch with events when timing is enabled.
struct LaunchTimer {
  rb_ctx* c;
  int fam;
  hipStream_t st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  LaunchTimer(rb_ctx* c_, int fam_, hipStream_t st_) : c(c_), fam(fam_), st(st_) {
    if (c && c->timing) {
      e0 = take_event(c);
      e1 = take_event(c);
      if (e0) (void)hipEventRecord(e0, st);
    }
  }
  ~LaunchTimer() {
    if (e0 && e1) {
      (void)hipEventRecord(e1, st);
      c->timed.push_back({fam, e0, e1});
    }
  }
};

template <int NP>
int launch_lu(const rb::NewtonF64Args& a, int it, hipStream_t st) {
  hipLaunchKernelGGL(rb::lu_f64_kernel<NP>, dim3((a.B + rb::kWaves - 1) / rb::kWaves),
                     dim3(rb::kThreads), 0, st, a, it);
  return RB_OK;
}

int dispatch_lu(int NP, const rb::NewtonF64Args& a, int it, hipStream_t st) {
  switch (NP) {
    case 8: return launch_lu<8>(a, it, st);
    case 16: return launch_lu<16>(a, it, st);
    case 24: return launch_lu<24>(a, it, st);
    case 32: return launch_lu<32>(a, it, st);
    case 40: return launch_lu<40>(a, it, st);
    case 48: return launch_lu<48>(a, it, st);
    case 56: return launch_lu<56>(a, it, st);
    case 64: return launch_lu<64>(a, it, st);
  }
  return fail(RB_E_UNSUPPORTED, "basis size bucket %d not built", NP);
}

// Enqueue a whole batched Newton solve: init, max_iter x (Jacobian kernel, LU kernel),
// final copy-out. Converged requests are skipped by both kernels through the done flags.
int enqueue_newton(rb_ctx* c, const rb::NewtonF64Args& a, hipStream_t st) {
  const int NP = a.s.NP;
  const int64_t Bp = (int64_t)(a.B + rb::kBT - 1) / rb::kBT * rb::kBT;
  const size_t lds = (size_t)rb::jac_lds_bytes(a.nks, NP);
  if (lds > 64 * 1024)
    HIP_TRY(hipFuncSetAttribute((const void*)rb::jac_f64_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(rb::newton_init_kernel, dim3(launch_grid(Bp * NP)), dim3(256), 0, st, a);
  for (int it = 0; it < a.maxit; ++it) {
    {
      LaunchTimer t(c, FAM_JACOBIAN, st);
      hipLaunchKernelGGL(rb::jac_f64_kernel, dim3(Bp / rb::kBT), dim3(rb::kThreads), lds, st,
                         a);
    }
    LaunchTimer t(c, FAM_LU, st);
    if (int rc = dispatch_lu(NP, a, it, st)) return rc;
  }
  hipLaunchKernelGGL(rb::newton_final_kernel, dim3(launch_grid((int64_t)a.B * a.ldu)),
                     dim3(256), 0, st, a);
  HIP_TRY(hipGetLastError());
  return RB_OK;
}

template <int NPP>
int launch_pressure(const rb::PressureF64Args& a, int NPU, hipStream_t st) {
  const size_t lds = (size_t)rb::pressure_lds_bytes(a.nks, NPU, NPP);
  if (lds > 64 * 1024)
    HIP_TRY(hipFuncSetAttribute((const void*)rb::pressure_f64_kernel<NPP>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const int grid = (a.B + rb::kBT - 1) / rb::kBT;
  hipLaunchKernelGGL(rb::pressure_f64_kernel<NPP>, dim3(grid), dim3(rb::kThreads), lds, st,
                     a, NPU);
  HIP_TRY(hipGetLastError());
  return RB_OK;
}

int dispatch_pressure(int NPP, const rb::PressureF64Args& a, int NPU, hipStream_t st) {
  switch (NPP) {
    case 8: return launch_pressure<8>(a, NPU, st);
    case 16: return launch_pressure<16>(a, NPU, st);
    case 24: return launch_pressure<24>(a, NPU, st);
    case 32: return launch_pressure<32>(a, NPU, st);
    case 40: return launch_pressure<40>(a, NPU, st);
    case 48: return launch_pressure<48>(a, NPU, st);
    case 56: return launch_pressure<56>(a, NPU, st);
    case 64: return launch_pressure<64>(a, NPU, st);
  }
  return fail(RB_E_UNSUPPORTED, "pressure size bucket %d not built", NPP);
}

}  // namespace

extern "C" {

const char* rb_last_error(void) { return g_err.c_str(); }

int rb_create(int device, size_t hbm_budget_bytes, rb_ctx** out) {
  if (!out) return fail(RB_E_INVAL, "rb_create: out is NULL");
  *out = nullptr;
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (device < 0 || device >= n)
    return fail(RB_E_INVAL, "rb_create: device %d not in [0, %d)", device, n);
  HIP_TRY(hipSetDevice(device));
  rb_ctx* c = new rb_ctx;
  c->device = device;
  c->budget = hbm_budget_bytes;
  *out = c;
  g_err.clear();
  return RB_OK;
}

int rb_destroy(rb_ctx* c) {
  if (!c) return fail(RB_E_INVAL, "rb_destroy: NULL context");
  (void)hipSetDevice(c->device);
  for (auto& sp : c->sets) {
    if (!sp) continue;
    Set& s = *sp;
    for (DevBuf* b : {&s.A, &s.C, &s.F, &s.H, &s.BpT, &s.Asv, &s.Csv, &s.Fs}) dev_free(c, *b);
    for (auto& kv : s.solve_f64) dev_free(c, kv.second.buf);
    for (auto& kv : s.press_f64) dev_free(c, kv.second.buf);
  }
  for (auto& kv : c->ws) dev_free(c, kv.second.buf);
  for (auto& t : c->timed) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (auto e : c->event_pool) (void)hipEventDestroy(e);
  delete c;
  return RB_OK;
}

size_t rb_hbm_used(const rb_ctx* c) { return c ? c->used : 0; }

int rb_load_tensors(rb_ctx* c, const rb_tensors_desc* d, int* set_id_out) {
  if (!c || !d || !set_id_out) return fail(RB_E_INVAL, "rb_load_tensors: NULL argument");
  if (d->N < 1 || d->N > RB_MAX_N)
    return fail(RB_E_INVAL, "rb_load_tensors: N=%d outside [1, %d]", d->N, RB_MAX_N);
  if (d->Q < 1 || d->Q > RB_MAX_Q || d->Qc < 1 || d->Qc > RB_MAX_QC || d->Qf < 1 ||
      d->Qf > RB_MAX_QF)
    return fail(RB_E_INVAL, "rb_load_tensors: term counts Q=%d Qc=%d Qf=%d out of range",
                d->Q, d->Qc, d->Qf);
  if (!d->A || !d->C || !d->F) return fail(RB_E_INVAL, "rb_load_tensors: A, C or F is NULL");
  if (d->Np < 0 || d->Np > RB_MAX_NP)
    return fail(RB_E_INVAL, "rb_load_tensors: Np=%d outside [0, %d]", d->Np, RB_MAX_NP);
  if (d->Np > 0 && (d->Qb < 1 || d->Qb > RB_MAX_QB || !d->Bp || !d->Asv || !d->Csv || !d->Fs))
    return fail(RB_E_INVAL, "rb_load_tensors: incomplete pressure data (Qb=%d)", d->Qb);
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc = use_device(c)) return rc;
  auto s = std::make_unique<Set>();
  const size_t N = d->N;
  s->N = d->N; s->Q = d->Q; s->Qc = d->Qc; s->Qf = d->Qf; s->Np = d->Np; s->Qb = d->Qb;
  int rc;
  auto cleanup = [&](int code) {
    for (DevBuf* b : {&s->A, &s->C, &s->F, &s->H, &s->BpT, &s->Asv, &s->Csv, &s->Fs})
      dev_free(c, *b);
    for (auto& kv : s->solve_f64) dev_free(c, kv.second.buf);
    for (auto& kv : s->press_f64) dev_free(c, kv.second.buf);
    return code;
  };
  if ((rc = upload(c, s->A, d->A, d->Q * N * N))) return cleanup(rc);
  if ((rc = upload(c, s->C, d->C, d->Qc * N * N * N))) return cleanup(rc);
  if ((rc = upload(c, s->F, d->F, d->Qf * N))) return cleanup(rc);
  if (d->H) {
    if ((rc = upload(c, s->H, d->H, N * N))) return cleanup(rc);
    s->hasH = true;
  }
  if (d->Np > 0) {
    const size_t P = d->Np;
    std::vector<double> bt(d->Qb * P * P);
    for (int q = 0; q < d->Qb; ++q)
      for (size_t i = 0; i < P; ++i)
        for (size_t j = 0; j < P; ++j) bt[(q * P + j) * P + i] = d->Bp[(q * P + i) * P + j];
    if ((rc = upload(c, s->BpT, bt.data(), bt.size()))) return cleanup(rc);
    if ((rc = upload(c, s->Asv, d->Asv, d->Q * P * N))) return cleanup(rc);
    if ((rc = upload(c, s->Csv, d->Csv, d->Qc * P * N * N))) return cleanup(rc);
    if ((rc = upload(c, s->Fs, d->Fs, d->Qf * P))) return cleanup(rc);
  }
  Pack* pk;
  if ((rc = solve_pack_f64(c, s.get(), d->N, &pk))) return cleanup(rc);
  if (d->Np > 0 && (rc = press_pack_f64(c, s.get(), d->N, d->Np, &pk))) return cleanup(rc);
  c->sets.push_back(std::move(s));
  *set_id_out = (int)c->sets.size() - 1;
  return RB_OK;
}

int rb_theta(rb_ctx* c, int set, int B, const double* mu, double* ta, double* tc, double* tf,
             double* tb, void* stream) {
  if (!c) return fail(RB_E_INVAL, "rb_theta: NULL context");
  Set* s = get_set(c, set);
  if (!s) return fail(RB_E_INVAL, "rb_theta: unknown set %d", set);
  if (B < 0) return fail(RB_E_INVAL, "rb_theta: B=%d", B);
  if (B == 0) return RB_OK;
  if (!mu || !ta || !tc || !tf) return fail(RB_E_INVAL, "rb_theta: NULL array");
  if (int rc = use_device(c)) return rc;
  hipLaunchKernelGGL(rb::theta_kernel, dim3((B + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, mu, B, s->Q, s->Qc, s->Qf, s->Np > 0 ? s->Qb : 1,
                     ta, tc, tf, s->Np > 0 ? tb : nullptr);
  HIP_TRY(hipGetLastError());
  return RB_OK;
}

int rb_solve_batch(rb_ctx* c, int set, int B, int N, int ldu, const double* ta,
                   const double* tc, const double* tf, const double* fover, const double* u0,
                   const rb_solve_opts* opts, double* u, int* iters, int* status,
                   void* stream) {
  if (!c) return fail(RB_E_INVAL, "rb_solve_batch: NULL context");
  Set* s = get_set(c, set);
  if (!s) return fail(RB_E_INVAL, "rb_solve_batch: unknown set %d", set);
  if (B < 0) return fail(RB_E_INVAL, "rb_solve_batch: B=%d", B);
  if (N < 1 || N > s->N)
    return fail(RB_E_INVAL, "rb_solve_batch: N=%d outside [1, %d]", N, s->N);
  if (ldu < N) return fail(RB_E_INVAL, "rb_solve_batch: ldu=%d < N=%d", ldu, N);
  rb_solve_opts o = {1e-12, 10, RB_PREC_F64, 1};
  if (opts) o = *opts;
  if (!(o.tol >= 0.0) || o.max_iter < 1 || o.max_iter > 1000)
    return fail(RB_E_INVAL, "rb_solve_batch: bad options (tol=%g, max_iter=%d)", o.tol,
                o.max_iter);
  if (o.precision != RB_PREC_F64)
    return fail(RB_E_UNSUPPORTED, "rb_solve_batch: precision %d not available", o.precision);
  if (B == 0) return RB_OK;
  if (!ta || !tc || (!tf && !fover) || !u || !iters || !status)
    return fail(RB_E_INVAL, "rb_solve_batch: NULL array");
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc = use_device(c)) return rc;
  Pack* pk;
  if (int rc = solve_pack_f64(c, s, N, &pk)) return rc;
  const int64_t mp = ceil_to((int64_t)N * N, 16);
  const int NP = np_bucket(N);
  const int64_t Bp = ceil_to(B, rb::kBT);
  Workspace* w;
  if (int rc = workspace(c, stream, newton_state_bytes(Bp, NP, mp), &w)) return rc;
  rb::NewtonF64Args a;
  a.op = (const double*)pk->buf.p;
  a.nrb = pk->nrb; a.nks_s = pk->nks_s; a.nks = pk->nks;
  a.N = N; a.Nm = s->N; a.Q = s->Q; a.Qc = s->Qc; a.Qf = s->Qf; a.B = B; a.ldu = ldu;
  a.maxit = o.max_iter; a.tol = o.tol;
  a.ta = ta; a.tc = tc; a.tf = tf; a.fover = fover; a.u0 = u0;
  a.F = (const double*)s->F.p;
  a.H = s->hasH ? (const double*)s->H.p : nullptr;
  a.u = u; a.iters = iters; a.status = status;
  a.s = carve_state(w->buf.p, Bp, NP, mp);
  return enqueue_newton(c, a, (hipStream_t)stream);
}

int rb_solve_uneven(rb_ctx* c, int, int, const int*, int, const double*, const double*,
                    const double*, const double*, const double*, const rb_solve_opts*,
                    double*, int*, int*, void*) {
  if (!c) return fail(RB_E_INVAL, "rb_solve_uneven: NULL context");
  return fail(RB_E_UNSUPPORTED, "rb_solve_uneven: not available in this build");
}

int rb_recover_pressure(rb_ctx* c, int set, int B, int N, int Np, int ldu, int ldp,
                        const double* ta, const double* tc, const double* tf,
                        const double* tb, const double* u, double* p, int* status,
                        void* stream) {
  if (!c) return fail(RB_E_INVAL, "rb_recover_pressure: NULL context");
  Set* s = get_set(c, set);
  if (!s) return fail(RB_E_INVAL, "rb_recover_pressure: unknown set %d", set);
  if (s->Np == 0) return fail(RB_E_INVAL, "rb_recover_pressure: set %d has no pressure data", set);
  if (B < 0) return fail(RB_E_INVAL, "rb_recover_pressure: B=%d", B);
  if (N < 1 || N > s->N || Np < 1 || Np > s->Np)
    return fail(RB_E_INVAL, "rb_recover_pressure: N=%d / Np=%d out of range", N, Np);
  if (ldu < N || ldp < Np)
    return fail(RB_E_INVAL, "rb_recover_pressure: ldu=%d / ldp=%d too small", ldu, ldp);
  if (B == 0) return RB_OK;
  if (!ta || !tc || !tf || !tb || !u || !p || !status)
    return fail(RB_E_INVAL, "rb_recover_pressure: NULL array");
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc = use_device(c)) return rc;
  Pack* pk;
  if (int rc = press_pack_f64(c, s, N, Np, &pk)) return rc;
  rb::PressureF64Args a;
  a.op = (const double*)pk->buf.p;
  a.nrb = pk->nrb; a.nks_s = pk->nks_s; a.nks = pk->nks;
  a.N = N; a.Np = Np; a.Nm = s->N; a.Npm = s->Np; a.Q = s->Q; a.Qc = s->Qc; a.Qf = s->Qf;
  a.Qb = s->Qb; a.B = B; a.ldu = ldu; a.ldp = ldp;
  a.ta = ta; a.tc = tc; a.tf = tf; a.tb = tb; a.u = u;
  a.BpT = (const double*)s->BpT.p;
  a.Fs = (const double*)s->Fs.p;
  a.p = p; a.status = status;
  LaunchTimer t(c, FAM_PRESSURE, (hipStream_t)stream);
  return dispatch_pressure(np_bucket(Np), a, N, (hipStream_t)stream);
}

int rb_timing_enable(rb_ctx* c, int enable) {
  if (!c) return fail(RB_E_INVAL, "rb_timing_enable: NULL context");
  std::lock_guard<std::mutex> lk(c->mu);
  c->timing = enable != 0;
  return RB_OK;
}

int rb_timing_read(rb_ctx* c, const char* family, double* total_ms, int* launches) {
  if (!c || !family || !total_ms || !launches)
    return fail(RB_E_INVAL, "rb_timing_read: NULL argument");
  int fam = -1;
  for (int i = 0; i < FAM_COUNT; ++i)
    if (std::strcmp(family, kFamilies[i]) == 0) fam = i;
  if (fam < 0) return fail(RB_E_INVAL, "rb_timing_read: unknown kernel family '%s'", family);
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc = use_device(c)) return rc;
  double tot = 0.0;
  int n = 0;
  std::vector<TimedLaunch> keep;
  for (auto& t : c->timed) {
    if (t.family != fam) {
      keep.push_back(t);
      continue;
    }
    HIP_TRY(hipEventSynchronize(t.stop));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, t.start, t.stop));
    tot += ms;
    ++n;
    c->event_pool.push_back(t.start);
    c->event_pool.push_back(t.stop);
  }
  c->timed.swap(keep);
  *total_ms = tot;
  *launches = n;
  return RB_OK;
}

}  // extern "C"
