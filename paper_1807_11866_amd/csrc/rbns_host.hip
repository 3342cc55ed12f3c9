// rbns_host.hip -- host side of the C ABI declared in include/rbns.h: contexts, HBM budget,
// resident tensor sets, packed operands, per-stream workspaces and kernel launches.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/rbns.h"
#include "rb_launch.hpp"
#include "rb_reconstruct.hpp"
#include "rb_assemble.hpp"

// Device scratch of rb_solve_batch_noalloc: the Newton state of one call lives here instead of
// in a per-stream workspace, so that entry point allocates nothing. Each device holds its own
// copy for the life of the process. In host code `scratch` names a host-side stand-in, never
// the device memory: kernels and copies get the per-device address that rb_create looks up
// with hipGetSymbolAddress (scratch_ptr below).
static __device__ __align__(256) char scratch[RB_NOALLOC_SCRATCH_BYTES];

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
  const void* lo = nullptr;  // BF16x3: low parts (inside buf)
  int nrb = 0, nks_s = 0, nks = 0;
  int nchunk = 1;          // tensor part = nchunk chunks of (nks - nks_s) / nchunk k-steps
  int naff = 0;            // long expansions: affine chunks of the same length (nks_s of them)
};

// Newton iteration counts of the FP64 batches of one basis size: the final kernel writes the
// batch's largest count straight into the pinned `host` word, and `ev` is recorded behind it;
// a later batch reads the word once the event has completed (never waiting for it) and runs
// that many regular iterations before the tail launch.
struct NewtonHist {
  int* host = nullptr;
  hipEvent_t ev = nullptr;
  bool pending = false;
  int k = 0;                               // learned count (0: none yet)
};

struct Set {
  int N = 0, Q = 0, Qc = 0, Qf = 0, Np = 0, Qb = 0;
  DevBuf A, C, F, H, BpT, Asv, Csv, Fs;
  bool hasH = false;
  std::map<int, Pack> solve_f64;                     // key: N
  std::map<std::pair<int, int>, Pack> press_f64;     // key: (N, Np)
  std::map<std::pair<int, int>, Pack> solve_lp;      // key: (N, RB_PREC_*)
  std::map<int, NewtonHist> hist;                    // key: N
};

struct Workspace {
  DevBuf buf;            // Newton state of the last batch on this stream (see NewtonState)
};

// Tile shape of one (set, N, precision, batch size class): row splits per 64-request tile of
// the contraction and the pivot-row broadcast of the one-wavefront FP64 LU.
struct Tune {
  int nsplit = 8;
  int lu = RB_LU_AUTO;
};

// A captured uneven-batch graph and the shape it was captured for.
struct GraphEntry {
  std::vector<int64_t> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t last = 0;
};

}  // namespace

struct TimedLaunch {
  int family;
  hipEvent_t start, stop;
};

struct rb_ctx {
  int device = 0;
  char* scratch = nullptr;              // this device's address of `scratch`
  size_t budget = 0, used = 0;
  std::vector<std::unique_ptr<Set>> sets;
  std::map<void*, Workspace> ws;
  std::mutex mu;
  bool timing = false;
  int lu = RB_LU_AUTO;                  // LU variant of the FP64 solves (RB_LU_*)
  std::vector<TimedLaunch> timed;       // recorded, not yet read
  std::vector<hipEvent_t> event_pool;
  // autotuner results: (set, N, precision, batch size class) -> tile shape
  std::map<std::tuple<int, int, int, int>, Tune> tune;
  bool autotune = true;
  bool uneven_graphs = true;            // capture and replay uneven-batch group chains
  int newton_k = -1;                    // FP64 regular iterations: -1 learned, 0 all, n > 0 n
  // uneven batches: pinned staging of the per-request sizes / permutation, capture streams,
  // graph cache and the shapes seen once (captured on their second occurrence)
  int* pin = nullptr;
  size_t pin_cap = 0;
  hipEvent_t pin_ev = nullptr;          // recorded after the last copy out of `pin`
  bool pin_busy = false;
  hipStream_t cap_stream = nullptr;
  std::vector<hipStream_t> branches;
  std::vector<GraphEntry> graphs;
  std::vector<std::vector<int64_t>> seen;
  uint64_t tick = 0;
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

// k-steps of a packed row block: affine part ceil(Q/4), tensor part ceil(Qc*N/4) split into
// nchunk <= 64-k-step chunks of an even length KC (the FP64 contraction is instantiated per
// even chunk length and holds one chunk of W in registers), zero padded.
void tensor_chunks(int Qc, int N, int* nchunk, int* kc) {
  const int raw = (int)(ceil_to((int64_t)Qc * N, 4) / 4);
  *nchunk = (raw + rb::kMaxKC - 1) / rb::kMaxKC;
  *kc = (int)ceil_to((raw + *nchunk - 1) / *nchunk, 2);
}
int tensor_ksteps(int Qc, int N) {
  int n, kc;
  tensor_chunks(Qc, N, &n, &kc);
  return n * kc;
}

// FP64 operand layout of basis size N: the affine part is padded to kAmax k-steps in front of
// the first tensor chunk when Q <= 4*kAmax, else it takes naff chunks of its own (long
// expansions); returns the affine k-steps.
int f64_layout(const Set* s, int N, int* nchunk, int* kc, int* naff) {
  tensor_chunks(s->Qc, N, nchunk, kc);
  if (s->Q <= 4 * rb::kAmax) {
    *naff = 0;
    return rb::kAmax;
  }
  const int ka = (s->Q + 3) / 4;
  *naff = (ka + *kc - 1) / *kc;
  return *naff * *kc;
}

int make_pack(rb_ctx* c, Set* s, int N, int R, bool solve, Pack* p) {
  p->nrb = (int)(ceil_to((int64_t)N * R, 16) / 16);
  int kc;
  p->nks_s = f64_layout(s, N, &p->nchunk, &kc, &p->naff);
  p->nks = p->nks_s + p->nchunk * kc;
  const int64_t total = (int64_t)p->nrb * p->nks * 64;
  int rc = dev_alloc(c, p->buf, total * sizeof(double));
  if (rc) return rc;
  if (solve)
    hipLaunchKernelGGL(rb::pack_f64<true>, dim3(launch_grid(total)), dim3(256), 0, 0,
                       (const double*)s->C.p, (const double*)s->A.p, s->N, s->N, N, N, s->Q,
                       s->Qc, p->nks_s, p->nrb, p->nks, (double*)p->buf.p);
  else
    hipLaunchKernelGGL(rb::pack_f64<false>, dim3(launch_grid(total)), dim3(256), 0, 0,
                       (const double*)s->Csv.p, (const double*)s->Asv.p, s->N, s->Np, N, R,
                       s->Q, s->Qc, p->nks_s, p->nrb, p->nks, (double*)p->buf.p);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipDeviceSynchronize());
  return RB_OK;
}

// Solve operand for basis size N (built once on the device, then cached).
int solve_pack_f64(rb_ctx* c, Set* s, int N, Pack** out) {
  auto it = s->solve_f64.find(N);
  if (it != s->solve_f64.end()) { *out = &it->second; return RB_OK; }
  Pack p;
  if (int rc = make_pack(c, s, N, N, true, &p)) return rc;
  *out = &s->solve_f64.emplace(N, p).first->second;
  return RB_OK;
}

int press_pack_f64(rb_ctx* c, Set* s, int N, int Np, Pack** out) {
  auto key = std::make_pair(N, Np);
  auto it = s->press_f64.find(key);
  if (it != s->press_f64.end()) { *out = &it->second; return RB_OK; }
  Pack p;
  if (int rc = make_pack(c, s, N, Np, false, &p)) return rc;
  *out = &s->press_f64.emplace(key, p).first->second;
  return RB_OK;
}

// Mixed-precision packed operand for basis size N (FP32, BF16 or BF16 hi + lo copy of the FP64
// tensors). FP32: ceil(Qc*N/4) k-steps rounded up to even (to a multiple of 4 beyond 64); BF16:
// ceil(Qc*N/32) k-steps of 32. The whole tensor part is held in registers.
int lp_tensor_ksteps(int Qc, int N, bool bf16) {
  if (bf16) return (int)(ceil_to((int64_t)Qc * N, 32) / 32);
  const int raw = (int)(ceil_to((int64_t)Qc * N, 4) / 4);
  return (int)ceil_to(raw, raw > 64 ? 4 : 2);
}

int solve_pack_lp(rb_ctx* c, Set* s, int N, int prec, Pack** out) {
  const bool bf16 = prec != RB_PREC_F32, x3 = prec == RB_PREC_BF16X3;
  auto key = std::make_pair(N, prec);
  auto it = s->solve_lp.find(key);
  if (it != s->solve_lp.end()) { *out = &it->second; return RB_OK; }
  Pack p;
  p.nrb = (int)(ceil_to((int64_t)N * N, 16) / 16);
  p.nks_s = bf16 ? 1 : (s->Q + 3) / 4;
  p.nks = p.nks_s + lp_tensor_ksteps(s->Qc, N, bf16);
  const int64_t total = (int64_t)p.nrb * p.nks * 64 * (bf16 ? 8 : 1);
  int rc = dev_alloc(c, p.buf, total * (bf16 ? 2 : 4) * (x3 ? 2 : 1));
  if (rc) return rc;
  if (x3) {
    p.lo = (const uint16_t*)p.buf.p + total;
    hipLaunchKernelGGL((rb::pack_lp<true, true>), dim3(launch_grid(total)), dim3(256), 0, 0,
                       (const double*)s->C.p, (const double*)s->A.p, s->N, N, s->Q, s->Qc,
                       p.nks_s, p.nrb, p.nks, p.buf.p);
  } else if (bf16)
    hipLaunchKernelGGL(rb::pack_lp<true>, dim3(launch_grid(total)), dim3(256), 0, 0,
                       (const double*)s->C.p, (const double*)s->A.p, s->N, N, s->Q, s->Qc,
                       p.nks_s, p.nrb, p.nks, p.buf.p);
  else
    hipLaunchKernelGGL(rb::pack_lp<false>, dim3(launch_grid(total)), dim3(256), 0, 0,
                       (const double*)s->C.p, (const double*)s->A.p, s->N, N, s->Q, s->Qc,
                       p.nks_s, p.nrb, p.nks, p.buf.p);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipDeviceSynchronize());
  *out = &s->solve_lp.emplace(key, p).first->second;
  return RB_OK;
}

int launch_rc(int rc, const char* what) {
  if (rc == 0) return RB_OK;
  if (rc == -5) return fail(RB_E_UNSUPPORTED, "%s: size not built", what);
  return fail(RB_E_DEVICE, "%s: launch failed: %s", what, hipGetErrorString(hipGetLastError()));
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
size_t newton_state_bytes(int64_t Bp, int NP, int64_t mp, int nsplit, bool f64_j) {
  return (size_t)((f64_j ? Bp * mp : 0) + (2 + nsplit) * Bp * NP + Bp) * sizeof(double) +
         (size_t)3 * Bp * sizeof(int) + 256;
}

rb::NewtonState carve_state(void* base, int64_t Bp, int NP, int64_t mp, int nsplit,
                            bool f64_j) {
  rb::NewtonState s;
  double* d = (double*)base;
  s.J = f64_j ? d : nullptr;
  d += f64_j ? Bp * mp : 0;
  s.U = d;
  d += Bp * NP;
  s.Fv = d;
  d += Bp * NP;
  s.Wv = d;
  d += nsplit * Bp * NP;
  s.dprev = d;
  d += Bp;
  int* ip = (int*)d;
  s.done = ip;
  s.iters = ip + Bp;
  s.status = ip + 2 * Bp;
  s.mp = mp;
  s.NP = NP;
  s.Bp = Bp;
  s.nsplit = nsplit;
  return s;
}

// Mixed-precision buffers (FP32 Jacobians and partial sums, FP64 residual partials).
size_t lp_extra_bytes(int64_t Bp, int NP, int64_t mp, int nsplit) {
  return (size_t)(Bp * mp + nsplit * Bp * NP + 64) * sizeof(float) + 512 +
         (size_t)nsplit * Bp * NP * sizeof(double);
}

// An FP64 Jacobian per request (the mixed precisions keep theirs in FP32).
bool needs_f64_j(int precision) { return precision == RB_PREC_F64; }

// Register row length of the LU kernels (Newton and pressure): even up to 64 (one wavefront
// per system; every padded column costs a pivot step and a column of updates), multiples of
// 8 beyond (one workgroup of ceil(NP/64) wavefronts per system).
int np_bucket(int n) { return (int)ceil_to(n, n <= 64 ? 2 : 8); }

// Workspace of one same-N batch (padded to Bp requests): Newton state plus, for the mixed
// precisions, the low-precision buffers.
size_t solve_bytes(const Set* s, int N, int64_t Bp, int nsplit, int precision) {
  const int NP = np_bucket(N);
  const int64_t mp = ceil_to((int64_t)N * N, 16);
  size_t b = newton_state_bytes(Bp, NP, mp, nsplit, needs_f64_j(precision));
  if (precision != RB_PREC_F64) b += lp_extra_bytes(Bp, NP, mp, nsplit);
  return (size_t)ceil_to((int64_t)b, 256);
}

enum { FAM_JACOBIAN = 0, FAM_LU = 1, FAM_PRESSURE = 2, FAM_RESIDUAL = 3, FAM_RECONSTRUCT = 4,
       FAM_STOKES = 5, FAM_COUNT = 6 };
const char* const kFamilies[FAM_COUNT] = {"jacobian", "lu", "pressure", "residual",
                                          "reconstruct", "stokes"};

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

// Iteration history of (set, N) for a batch on stream st, created on first use; nullptr when
// the stream is being captured (no allocation, no event record) or the resources are missing
// (the schedule then keeps all max_iter regular iterations).
NewtonHist* newton_hist(rb_ctx* c, Set* s, int N, hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return nullptr;
  NewtonHist& h = s->hist[N];
  if (!h.ev) {
    if (hipHostMalloc((void**)&h.host, sizeof(int), hipHostMallocDefault) != hipSuccess) {
      h.host = nullptr;
      return nullptr;
    }
    if (hipEventCreateWithFlags(&h.ev, hipEventDisableTiming) != hipSuccess) {
      h.ev = nullptr;
      return nullptr;
    }
  }
  if (h.pending && hipEventQuery(h.ev) == hipSuccess) {
    h.k = *h.host;
    h.pending = false;
  }
  if (c->newton_k > 0) h.k = c->newton_k;
  return &h;
}

// Enqueue a whole batched Newton solve: init, the regular iterations (Jacobian kernel, LU
// kernel; without initial iterates the first Jacobian is A(mu), assembled from the affine
// operators alone), the tail launch for any further iterations, final copy-out. Converged
// requests are skipped by every kernel through the done flags. With a history h whose
// learned count K is below max_iter and the readlane LU, K regular iterations run and the
// tail takes the rest (the iterates are the same either way); otherwise all max_iter
// iterations are regular.
int enqueue_newton(rb_ctx* c, const rb::NewtonF64Args& a_in, int lu, hipStream_t st,
                   NewtonHist* h = nullptr) {
  rb::NewtonF64Args a = a_in;
  a.max_iters = h ? h->host : nullptr;
  const int NP = a.s.NP;
  const int64_t Bp = a.s.Bp;
  rb::ContractArgs g;
  g.op = a.op;
  g.nrb = a.nrb; g.nks = a.nks; g.kA = a.nks_s; g.nchunk = a.nchunk; g.naff = a.naff;
  g.nsplit = a.s.nsplit;
  g.R = a.N; g.N = a.N; g.M = a.N * a.N;
  g.Q = a.Q; g.Qc = a.Qc; g.B = a.B; g.Bp = Bp;
  g.ta = a.ta; g.tc = a.tc;
  g.U = a.s.U; g.ldU = NP;
  g.done = a.s.done;
  g.J = a.s.J; g.mp = a.s.mp;
  g.part = a.s.Wv; g.ldp = NP;
  int K = a.maxit;
  if (h && h->k > 0 && h->k < a.maxit &&
      rb::launch::lu_f64_variant(NP, a.N, lu) == RB_LU_READLANE)
    K = h->k;
  hipLaunchKernelGGL(rb::newton_init_kernel, dim3(launch_grid(Bp * NP)), dim3(256), 0, st, a);
  for (int it = 0; it < K; ++it) {
    if (it == 0 && !a.u0) {                // from u = 0: J = A(mu), A(mu) u = 0
      LaunchTimer t(c, FAM_STOKES, st);
      hipLaunchKernelGGL(rb::stokes_jacobian_kernel, rb::stokes_grid(a.B, a.N), dim3(256), 0,
                         st, a);
      HIP_TRY(hipGetLastError());
    } else {
      LaunchTimer t(c, FAM_JACOBIAN, st);
      if (int rc = launch_rc(rb::launch::contract_f64(rb::kModeJac, g, st), "jacobian")) return rc;
    }
    LaunchTimer t(c, FAM_LU, st);
    if (int rc = launch_rc(rb::launch::lu_f64(NP, a, it, lu, st), "lu")) return rc;
  }
  if (K < a.maxit) {
    LaunchTimer t(c, FAM_LU, st);
    if (int rc = launch_rc(rb::launch::newton_tail_f64(NP, g, a, K, st), "newton tail")) return rc;
  }
  hipLaunchKernelGGL(rb::newton_final_kernel, dim3(launch_grid((int64_t)a.B * a.ldu)),
                     dim3(256), 0, st, a);
  HIP_TRY(hipGetLastError());
  if (h) {
    HIP_TRY(hipEventRecord(h->ev, st));
    h->pending = true;
  }
  return RB_OK;
}

// Mixed-precision batched Newton: the low-precision phase (FP32, BF16 or BF16x3 contraction,
// FP32 LU, FP64 iterates) until each request's update is below tol or has stagnated, then up to
// refine_steps refinement steps, each with the FP64 residual and the Jacobian of the last
// low-precision step, until the update is below tol.
int enqueue_newton_lp(rb_ctx* c, Set* s, const rb::NewtonF64Args& a, int prec, int refine,
                      char* base, hipStream_t st) {
  const int N = a.N, NP = a.s.NP;
  const int64_t Bp = a.s.Bp, mp = a.s.mp;
  Pack *pf, *pl;
  if (int rc = solve_pack_f64(c, s, N, &pf)) return rc;
  if (int rc = solve_pack_lp(c, s, N, prec, &pl)) return rc;
  const int nsplit = a.s.nsplit;
  float* J32 = (float*)base;               // low-precision buffers (lp_extra_bytes)
  float* part32 = J32 + Bp * mp;
  double* partA = (double*)(part32 + nsplit * Bp * NP + 64);
  partA = (double*)(((uintptr_t)partA + 255) & ~(uintptr_t)255);

  rb::ContractLpArgs gl;
  gl.op = pl->buf.p; gl.op_lo = pl->lo;
  gl.nrb = pl->nrb; gl.kA = pl->nks_s; gl.nks = pl->nks;
  gl.N = N; gl.M = N * N; gl.Q = a.Q; gl.Qc = a.Qc; gl.B = a.B; gl.Bp = Bp;
  gl.ta = a.ta; gl.tc = a.tc; gl.U = a.s.U; gl.ldU = NP;
  gl.done = a.s.done;
  gl.J = J32; gl.mp = mp;
  gl.part = part32; gl.ldp = NP; gl.nsplit = nsplit;
  const int KT = pl->nks - pl->nks_s;

  rb::ContractArgs gr;                      // FP64 residual
  gr.op = (const double*)pf->buf.p;
  gr.nrb = pf->nrb; gr.nks = pf->nks; gr.kA = pf->nks_s; gr.nchunk = pf->nchunk;
  gr.naff = pf->naff;
  gr.nsplit = nsplit;
  gr.R = N; gr.N = N; gr.M = N * N;
  gr.Q = a.Q; gr.Qc = a.Qc; gr.B = a.B; gr.Bp = Bp;
  gr.ta = a.ta; gr.tc = a.tc; gr.U = a.s.U; gr.ldU = NP;
  gr.done = a.s.done; gr.J = nullptr; gr.mp = 0;
  gr.part = partA; gr.ldp = NP;

  rb::LpNewtonArgs la;
  la.N = N; la.Nm = a.Nm; la.B = a.B;
  la.tol = a.tol; la.H = a.H;
  la.stag = prec == RB_PREC_BF16 ? 5e-2 : 1e-3;
  la.J = J32; la.mp = mp; la.part = part32; la.partA = partA; la.nreq = a.nreq;
  la.s = a.s;

  hipLaunchKernelGGL(rb::newton_init_kernel, dim3(launch_grid(Bp * NP)), dim3(256), 0, st, a);
  for (int it = 0; it < a.maxit; ++it) {
    if (it == 0 && !a.u0) {                // from u = 0: J = A(mu), A(mu) u = 0
      LaunchTimer t(c, FAM_STOKES, st);
      hipLaunchKernelGGL(rb::stokes_jacobian_lp_kernel, rb::stokes_grid(a.B, N), dim3(256), 0,
                         st, a, J32, mp, part32, nsplit);
      HIP_TRY(hipGetLastError());
    } else {
      LaunchTimer t(c, FAM_JACOBIAN, st);
      if (int rc = launch_rc(rb::launch::contract_lp(prec, KT, gl, st), "lp jacobian")) return rc;
    }
    LaunchTimer t(c, FAM_LU, st);
    if (int rc = launch_rc(rb::launch::lu_lp(NP, false, la, it, st), "lp lu")) return rc;
  }
  if (refine > 0)
    hipLaunchKernelGGL(rb::lp_refine_reset_kernel, dim3(launch_grid(Bp)), dim3(256), 0, st,
                       a.B, Bp, a.s.done, a.s.status, a.s.dprev);
  for (int r = 0; r < refine; ++r) {
    {
      LaunchTimer t(c, FAM_RESIDUAL, st);
      if (int rc = launch_rc(rb::launch::contract_f64(rb::kModeResid, gr, st), "fp64 residual"))
        return rc;
    }
    LaunchTimer t(c, FAM_LU, st);
    if (int rc = launch_rc(rb::launch::lu_lp(NP, true, la, a.maxit + r, st), "lp refine")) return rc;
  }
  hipLaunchKernelGGL(rb::newton_final_kernel, dim3(launch_grid((int64_t)a.B * a.ldu)),
                     dim3(256), 0, st, a);
  HIP_TRY(hipGetLastError());
  return RB_OK;
}

int default_nsplit(int64_t Bp, int nrows);

// Row splits of a pressure recovery of B requests: `nsplit`, or 0 for the default of the
// batch size.
int pressure_nsplit(int B, int N, int Np, int nsplit) {
  return nsplit > 0 ? nsplit : default_nsplit(ceil_to(B, rb::kTile), Np * N);
}

size_t pressure_bytes(int B, int N, int Np, int nsplit = 0) {
  const int64_t Bp = ceil_to(B, rb::kTile);
  return (size_t)pressure_nsplit(B, N, Np, nsplit) * Bp * np_bucket(Np) * sizeof(double);
}

// Pressure recovery of B requests at (N, Np) (eqn sup-vvar): the pressure-operand
// contraction (A_sv u + C_sv(u,u), partial sums of `nsplit` row splits (0: the default) at
// `part`, pressure_bytes long) and the pivoted LU solve B(mu) p = f_s - A_sv u - C_sv(u,u).
int enqueue_pressure(rb_ctx* c, Set* s, int B, int N, int Np, int ldu, int ldp,
                     const double* ta, const double* tc, const double* tf, const double* tb,
                     const double* u, double* p, int* status, char* part, hipStream_t st,
                     int nsplit = 0) {
  Pack* pk;
  if (int rc = press_pack_f64(c, s, N, Np, &pk)) return rc;
  const int NPP = np_bucket(Np);
  const int64_t Bp = ceil_to(B, rb::kTile);
  rb::ContractArgs g;
  g.op = (const double*)pk->buf.p;
  g.nrb = pk->nrb; g.nks = pk->nks; g.kA = pk->nks_s; g.nchunk = pk->nchunk;
  g.naff = pk->naff;
  g.R = Np; g.N = N; g.M = Np * N;
  g.Q = s->Q; g.Qc = s->Qc; g.B = B; g.Bp = Bp;
  g.ta = ta; g.tc = tc;
  g.U = u; g.ldU = ldu;
  g.done = nullptr;
  g.J = nullptr; g.mp = 0;
  g.part = (double*)part; g.ldp = NPP; g.nsplit = pressure_nsplit(B, N, Np, nsplit);
  rb::PressureF64Args a;
  a.Np = Np; a.Npm = s->Np; a.Qf = s->Qf; a.Qb = s->Qb; a.B = B; a.ldp = ldp; a.Bp = Bp;
  a.tf = tf; a.tb = tb;
  a.BpT = (const double*)s->BpT.p;
  a.Fs = (const double*)s->Fs.p;
  a.part = g.part; a.nsplit = g.nsplit; a.ldpart = NPP;
  a.p = p; a.status = status;
  LaunchTimer t(c, FAM_PRESSURE, st);
  if (int rc = launch_rc(rb::launch::contract_f64(rb::kModePressure, g, st), "pressure"))
    return rc;
  if (int rc = launch_rc(rb::launch::plu_f64(NPP, a, c->lu, st), "pressure lu")) return rc;
  HIP_TRY(hipGetLastError());
  return RB_OK;
}

// Shape class of a batch for the tuning table: ceil(log2(tiles)).
int batch_class(int64_t Bp) {
  int t = 0;
  while (((int64_t)rb::kTile << t) < Bp) ++t;
  return t;
}

// Row splits per 64-request tile when no tuned shape is recorded: 8 (one per XCD, so each
// XCD's L2 holds an eighth of the operand) for batches that fill the chip, more for small
// batches so that about 512 workgroups still run, at least 4 row blocks per split.
int default_nsplit(int64_t Bp, int nrows) {
  const int64_t tiles = std::max<int64_t>(1, Bp / rb::kTile);
  int want = rb::kSplit;
  while (want < rb::kMaxSplit && tiles * want < 512) want *= 2;
  const int nrb = (nrows + 15) / 16;
  return std::max(1, std::min({want, std::max(rb::kSplit, nrb / 4), nrb}));
}

// Partial-sum slots a state region reserves so that the autotuner can try every candidate.
int region_nsplit(int64_t Bp, int N) { return std::max(16, default_nsplit(Bp, N * N)); }

Tune tune_for(rb_ctx* c, int set, int N, int precision, int64_t Bp) {
  auto it = c->tune.find(std::make_tuple(set, N, precision, batch_class(Bp)));
  if (it != c->tune.end()) return it->second;
  Tune t;
  t.nsplit = default_nsplit(Bp, N * N);
  t.lu = c->lu;
  return t;
}

// The low-precision contraction keeps the trigonometric theta lists in registers: long
// expansions run in FP64 only.
int check_lp_terms(const char* fn, const Set* s, const rb_solve_opts& o) {
  if (o.precision != RB_PREC_F64 && (s->Q > rb::kMaxQ || s->Qc > rb::kMaxQc))
    return fail(RB_E_UNSUPPORTED, "%s: mixed precision takes Q <= %d and Qc <= %d (Q=%d Qc=%d)",
                fn, rb::kMaxQ, rb::kMaxQc, s->Q, s->Qc);
  return RB_OK;
}

int check_opts(const char* fn, const rb_solve_opts& o) {
  if (!(o.tol >= 0.0) || o.max_iter < 1 || o.max_iter > 1000)
    return fail(RB_E_INVAL, "%s: bad options (tol=%g, max_iter=%d)", fn, o.tol, o.max_iter);
  if (o.precision != RB_PREC_F64 && o.precision != RB_PREC_F32 && o.precision != RB_PREC_BF16 &&
      o.precision != RB_PREC_BF16X3)
    return fail(RB_E_INVAL, "%s: unknown precision %d", fn, o.precision);
  if (o.precision != RB_PREC_F64 && (o.refine_steps < 0 || o.refine_steps > 100))
    return fail(RB_E_INVAL, "%s: refine_steps=%d", fn, o.refine_steps);
  return RB_OK;
}

// Newton arguments of one same-N batch whose state lives at `region` (solve_bytes long).
rb::NewtonF64Args make_args(Set* s, Pack* pk, int N, int B, int ldu, const rb_solve_opts& o,
                            const double* ta, const double* tc, const double* tf,
                            const double* fover, const double* u0, double* u, int* iters,
                            int* status, char* region, int nsplit,
                            const int* nreq = nullptr) {
  rb::NewtonF64Args a;
  a.op = (const double*)pk->buf.p;
  a.nrb = pk->nrb; a.nks_s = pk->nks_s; a.nks = pk->nks; a.nchunk = pk->nchunk;
  a.naff = pk->naff;
  a.N = N; a.Nm = s->N; a.Q = s->Q; a.Qc = s->Qc; a.Qf = s->Qf; a.B = B; a.ldu = ldu;
  a.maxit = o.max_iter; a.tol = o.tol;
  a.ta = ta; a.tc = tc; a.tf = tf; a.fover = fover; a.u0 = u0; a.nreq = nreq;
  a.F = (const double*)s->F.p;
  a.H = s->hasH ? (const double*)s->H.p : nullptr;
  a.u = u; a.iters = iters; a.status = status; a.max_iters = nullptr;
  const int64_t Bp = ceil_to(B, rb::kTile);
  a.s = carve_state(region, Bp, np_bucket(N), ceil_to((int64_t)N * N, 16), nsplit,
                    needs_f64_j(o.precision));
  return a;
}

int enqueue_solve(rb_ctx* c, Set* s, const rb::NewtonF64Args& a, const rb_solve_opts& o,
                  const Tune& t, char* region, hipStream_t st, NewtonHist* h = nullptr) {
  if (o.precision == RB_PREC_F64) return enqueue_newton(c, a, t.lu, st, h);
  char* lp = region + newton_state_bytes(a.s.Bp, a.s.NP, a.s.mp, a.s.nsplit,
                                        needs_f64_j(o.precision));
  return enqueue_newton_lp(c, s, a, o.precision, o.refine_steps, lp, st);
}

// Autotuner. On the batch at hand (its state region sized for region_nsplit partials), time
// the first Newton contraction for each row-split count and, for the one-wavefront FP64 LU,
// both pivot-row broadcasts; record the fastest shape for (set, N, precision, batch class).
// Synchronous on st; must not run under stream capture.
int autotune_batch(rb_ctx* c, Set* s, int set, rb::NewtonF64Args a, const rb_solve_opts& o,
                   char* region, hipStream_t st, Tune* out) {
  const int N = a.N, NP = a.s.NP;
  const int64_t Bp = a.s.Bp, mp = a.s.mp;
  const bool lp = o.precision != RB_PREC_F64;
  Pack* pl = nullptr;
  if (lp)
    if (int rc = solve_pack_lp(c, s, N, o.precision, &pl)) return rc;
  hipEvent_t e0 = take_event(c), e1 = take_event(c);
  if (!e0 || !e1) return fail(RB_E_DEVICE, "autotune: cannot create events");
  auto release = [&](int rc) {
    c->event_pool.push_back(e0);
    c->event_pool.push_back(e1);
    return rc;
  };
  const int rsplit = region_nsplit(Bp, N);
  a.s = carve_state(region, Bp, NP, mp, rsplit, needs_f64_j(o.precision));
  char* lpb = region + newton_state_bytes(Bp, NP, mp, rsplit, needs_f64_j(o.precision));
  auto contract = [&](int nsplit) -> int {
    a.s.nsplit = nsplit;
    if (!lp) {
      rb::ContractArgs g;
      g.op = a.op;
      g.nrb = a.nrb; g.nks = a.nks; g.kA = a.nks_s; g.nchunk = a.nchunk; g.naff = a.naff;
      g.nsplit = nsplit;
      g.R = N; g.N = N; g.M = N * N;
      g.Q = a.Q; g.Qc = a.Qc; g.B = a.B; g.Bp = Bp;
      g.ta = a.ta; g.tc = a.tc; g.U = a.s.U; g.ldU = NP;
      g.done = a.s.done; g.J = a.s.J; g.mp = mp;
      g.part = a.s.Wv; g.ldp = NP;
      return launch_rc(rb::launch::contract_f64(rb::kModeJac, g, st), "autotune contraction");
    }
    rb::ContractLpArgs g;
    g.op = pl->buf.p; g.op_lo = pl->lo;
    g.nrb = pl->nrb; g.kA = pl->nks_s; g.nks = pl->nks;
    g.N = N; g.M = N * N; g.Q = a.Q; g.Qc = a.Qc; g.B = a.B; g.Bp = Bp;
    g.ta = a.ta; g.tc = a.tc; g.U = a.s.U; g.ldU = NP;
    g.done = a.s.done; g.J = (float*)lpb; g.mp = mp;
    g.part = (float*)lpb + Bp * mp; g.ldp = NP; g.nsplit = nsplit;
    return launch_rc(rb::launch::contract_lp(o.precision, pl->nks - pl->nks_s, g, st),
                     "autotune contraction");
  };
  auto timed = [&](auto&& launch, float* ms) -> int {
    for (int rep = 0; rep < 2; ++rep) {          // the second run is timed
      HIP_TRY(hipEventRecord(e0, st));
      if (int rc = launch()) return rc;
      HIP_TRY(hipEventRecord(e1, st));
    }
    HIP_TRY(hipEventSynchronize(e1));
    HIP_TRY(hipEventElapsedTime(ms, e0, e1));
    return RB_OK;
  };
  hipLaunchKernelGGL(rb::newton_init_kernel, dim3(launch_grid(Bp * NP)), dim3(256), 0, st, a);
  Tune best;
  best.lu = c->lu;
  float best_ms = 1e30f;
  for (int ns : {2, 4, 8, 16, default_nsplit(Bp, N * N)}) {
    if (ns > rsplit || ns > a.nrb) continue;   // no slots / more splits than row blocks
    float ms = 0.f;
    if (int rc = timed([&] { return contract(ns); }, &ms)) return release(rc);
    if (ms < best_ms) {
      best_ms = ms;
      best.nsplit = ns;
    }
  }
  if (!lp && NP <= 64) {
    float lu_best = 1e30f;
    for (int v : {RB_LU_READLANE, RB_LU_LDS, RB_LU_MFMA}) {
      if (v == RB_LU_MFMA && N > RB_LU_MFMA_MAX_N) continue;
      hipLaunchKernelGGL(rb::newton_init_kernel, dim3(launch_grid(Bp * NP)), dim3(256), 0, st, a);
      if (int rc = contract(best.nsplit)) return release(rc);
      float ms = 0.f;
      if (int rc = timed([&] { return launch_rc(rb::launch::lu_f64(NP, a, 0, v, st),
                                                "autotune lu"); }, &ms))
        return release(rc);
      if (ms < lu_best) {
        lu_best = ms;
        best.lu = v;
      }
    }
  }
  c->tune[std::make_tuple(set, N, o.precision, batch_class(Bp))] = best;
  *out = best;
  return release(RB_OK);
}

// The pinned staging buffer is shared by every stream of the context: an uneven call's
// asynchronous copy of the permutation out of it may still be pending on another stream, so
// wait for that copy before the buffer is rewritten or replaced.
int ensure_pinned(rb_ctx* c, size_t ints) {
  if (c->pin_busy) {
    HIP_TRY(hipEventSynchronize(c->pin_ev));
    c->pin_busy = false;
  }
  if (c->pin_cap >= ints) return RB_OK;
  if (c->pin) HIP_TRY(hipHostFree(c->pin));
  c->pin = nullptr;
  c->pin_cap = 0;
  HIP_TRY(hipHostMalloc((void**)&c->pin, ints * sizeof(int), hipHostMallocDefault));
  c->pin_cap = ints;
  return RB_OK;
}

int pin_release(rb_ctx* c, hipStream_t st) {
  if (!c->pin_ev) HIP_TRY(hipEventCreateWithFlags(&c->pin_ev, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(c->pin_ev, st));
  c->pin_busy = true;
  return RB_OK;
}

int ensure_streams(rb_ctx* c, int n) {
  if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  while ((int)c->branches.size() < n) {
    hipStream_t b;
    HIP_TRY(hipStreamCreateWithFlags(&b, hipStreamNonBlocking));
    c->branches.push_back(b);
  }
  return RB_OK;
}

// Device address of `scratch` on `device` (which must be current): looked up once per device
// and kept, since every device holds the array at its own address.
std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;

int scratch_address(int device, char** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(RB_E_DEVICE, "rb_create: no device address for the scratch array: %s",
                  hipGetErrorString(e));
    it = g_scratch_ptr.emplace(device, (char*)p).first;
  }
  *out = it->second;
  return RB_OK;
}

constexpr int kBranches = 4;      // concurrent bucket chains inside an uneven-batch graph
constexpr size_t kGraphCache = 16;

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
  char* sp = nullptr;
  if (int rc = scratch_address(device, &sp)) return rc;
  rb_ctx* c = new rb_ctx;
  c->device = device;
  c->scratch = sp;
  c->budget = hbm_budget_bytes;
  if (const char* v = getenv("RB_LU")) {
    if (strcmp(v, "auto") == 0) c->lu = RB_LU_AUTO;
    else if (strcmp(v, "readlane") == 0) c->lu = RB_LU_READLANE;
    else if (strcmp(v, "lds") == 0) c->lu = RB_LU_LDS;
    else if (strcmp(v, "mfma") == 0) c->lu = RB_LU_MFMA;
  }
  if (const char* v = getenv("RB_AUTOTUNE")) c->autotune = (strcmp(v, "0") != 0);
  if (const char* v = getenv("RB_UNEVEN_GRAPHS")) c->uneven_graphs = (strcmp(v, "0") != 0);
  if (const char* v = getenv("RB_NEWTON_K")) c->newton_k = atoi(v) < 0 ? -1 : atoi(v);
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
    for (auto& kv : s.solve_lp) dev_free(c, kv.second.buf);
    for (auto& kv : s.hist) {
      NewtonHist& h = kv.second;
      if (h.ev) {
        (void)hipEventSynchronize(h.ev);
        (void)hipEventDestroy(h.ev);
      }
      if (h.host) (void)hipHostFree(h.host);
    }
  }
  for (auto& kv : c->ws) dev_free(c, kv.second.buf);
  for (auto& t : c->timed) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (auto e : c->event_pool) (void)hipEventDestroy(e);
  for (auto& g : c->graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  for (auto b : c->branches) (void)hipStreamDestroy(b);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->pin_ev) {
    (void)hipEventSynchronize(c->pin_ev);
    (void)hipEventDestroy(c->pin_ev);
  }
  if (c->pin) (void)hipHostFree(c->pin);
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
  if (int rc = check_opts("rb_solve_batch", o)) return rc;
  if (int rc = check_lp_terms("rb_solve_batch", s, o)) return rc;
  if (o.precision == RB_PREC_F64 && N > RB_MAX_N_F64)
    return fail(RB_E_UNSUPPORTED, "rb_solve_batch: FP64 solves take N <= %d (N=%d)",
                RB_MAX_N_F64, N);
  if (B == 0) return RB_OK;
  if (!ta || !tc || (!tf && !fover) || !u || !iters || !status)
    return fail(RB_E_INVAL, "rb_solve_batch: NULL array");
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc = use_device(c)) return rc;
  Pack* pk;
  if (int rc = solve_pack_f64(c, s, N, &pk)) return rc;
  const int64_t Bp = ceil_to(B, rb::kTile);
  const Tune t = tune_for(c, set, N, o.precision, Bp);
  Workspace* w;
  if (int rc = workspace(c, stream, solve_bytes(s, N, Bp, t.nsplit, o.precision), &w))
    return rc;
  char* region = (char*)w->buf.p;
  rb::NewtonF64Args a = make_args(s, pk, N, B, ldu, o, ta, tc, tf, fover, u0, u, iters, status,
                                  region, t.nsplit);
  NewtonHist* h = (o.precision == RB_PREC_F64 && c->newton_k != 0)
                      ? newton_hist(c, s, N, (hipStream_t)stream)
                      : nullptr;
  return enqueue_solve(c, s, a, o, t, region, (hipStream_t)stream, h);
}

int rb_solve_batch_noalloc(rb_ctx* c, int set, int B, int N, int ldu, const double* ta,
                           const double* tc, const double* tf, const double* fover,
                           const double* u0, const rb_solve_opts* opts, double* u, int* iters,
                           int* status, void* stream) {
  if (!c) return fail(RB_E_INVAL, "rb_solve_batch_noalloc: NULL context");
  Set* s = get_set(c, set);
  if (!s) return fail(RB_E_INVAL, "rb_solve_batch_noalloc: unknown set %d", set);
  if (B < 0) return fail(RB_E_INVAL, "rb_solve_batch_noalloc: B=%d", B);
  if (N < 1 || N > s->N)
    return fail(RB_E_INVAL, "rb_solve_batch_noalloc: N=%d outside [1, %d]", N, s->N);
  if (ldu < N) return fail(RB_E_INVAL, "rb_solve_batch_noalloc: ldu=%d < N=%d", ldu, N);
  rb_solve_opts o = {1e-12, 10, RB_PREC_F64, 1};
  if (opts) o = *opts;
  if (int rc = check_opts("rb_solve_batch_noalloc", o)) return rc;
  if (int rc = check_lp_terms("rb_solve_batch_noalloc", s, o)) return rc;
  if (o.precision == RB_PREC_F64 && N > RB_MAX_N_F64)
    return fail(RB_E_UNSUPPORTED, "rb_solve_batch_noalloc: FP64 solves take N <= %d (N=%d)",
                RB_MAX_N_F64, N);
  if (B == 0) return RB_OK;
  if (!ta || !tc || (!tf && !fover) || !u || !iters || !status)
    return fail(RB_E_INVAL, "rb_solve_batch_noalloc: NULL array");
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc = use_device(c)) return rc;
  // The packed operands are built (allocated) by rb_load_tensors for the set's N in FP64 and
  // by the first rb_solve_batch / rb_autotune at any other (N, precision); this entry point
  // only uses them.
  auto pf = s->solve_f64.find(N);
  if (pf == s->solve_f64.end() ||
      (o.precision != RB_PREC_F64 && !s->solve_lp.count(std::make_pair(N, o.precision))))
    return fail(RB_E_STATE,
                "rb_solve_batch_noalloc: no packed operand for N=%d, precision %d yet (one "
                "rb_solve_batch call at that N and precision builds it)", N, o.precision);
  const int64_t Bp = ceil_to(B, rb::kTile);
  const Tune t = tune_for(c, set, N, o.precision, Bp);
  const size_t need = solve_bytes(s, N, Bp, t.nsplit, o.precision);
  if (need > (size_t)RB_NOALLOC_SCRATCH_BYTES)
    return fail(RB_E_NOMEM,
                "rb_solve_batch_noalloc: B=%d at N=%d needs %zu bytes of scratch, the device "
                "array holds %zu", B, N, need, (size_t)RB_NOALLOC_SCRATCH_BYTES);
  char* region = c->scratch;
  rb::NewtonF64Args a = make_args(s, &pf->second, N, B, ldu, o, ta, tc, tf, fover, u0, u,
                                  iters, status, region, t.nsplit);
  // no kernel timing here: its events are created on demand
  const bool timing = c->timing;
  c->timing = false;
  const int rc = enqueue_solve(c, s, a, o, t, region, (hipStream_t)stream);
  c->timing = timing;
  return rc;
}

int rb_autotune(rb_ctx* c, int set, int B, int N, const double* ta, const double* tc,
                const double* tf, const rb_solve_opts* opts, void* stream) {
  if (!c) return fail(RB_E_INVAL, "rb_autotune: NULL context");
  Set* s = get_set(c, set);
  if (!s) return fail(RB_E_INVAL, "rb_autotune: unknown set %d", set);
  if (B < 1 || N < 1 || N > s->N) return fail(RB_E_INVAL, "rb_autotune: B=%d N=%d", B, N);
  rb_solve_opts o = {1e-12, 10, RB_PREC_F64, 1};
  if (opts) o = *opts;
  if (int rc = check_opts("rb_autotune", o)) return rc;
  if (int rc = check_lp_terms("rb_autotune", s, o)) return rc;
  if (o.precision == RB_PREC_F64 && N > RB_MAX_N_F64)
    return fail(RB_E_UNSUPPORTED, "rb_autotune: FP64 solves take N <= %d", RB_MAX_N_F64);
  if (!ta || !tc || !tf) return fail(RB_E_INVAL, "rb_autotune: NULL array");
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc = use_device(c)) return rc;
  Pack* pk;
  if (int rc = solve_pack_f64(c, s, N, &pk)) return rc;
  const int64_t Bp = ceil_to(B, rb::kTile);
  Workspace* w;
  if (int rc = workspace(c, stream, solve_bytes(s, N, Bp, region_nsplit(Bp, N), o.precision), &w))
    return rc;
  char* region = (char*)w->buf.p;
  rb::NewtonF64Args a = make_args(s, pk, N, B, N, o, ta, tc, tf, nullptr, nullptr, nullptr,
                                  nullptr, nullptr, region, region_nsplit(Bp, N));
  Tune t;
  return autotune_batch(c, s, set, a, o, region, (hipStream_t)stream, &t);
}

int rb_tuned_config(rb_ctx* c, int set, int N, int precision, int B, int* nsplit,
                    int* lu_variant) {
  if (!c || !nsplit || !lu_variant) return fail(RB_E_INVAL, "rb_tuned_config: NULL argument");
  std::lock_guard<std::mutex> lk(c->mu);
  const Tune t = tune_for(c, set, N, precision, ceil_to(B < 1 ? 1 : B, rb::kTile));
  *nsplit = t.nsplit;
  *lu_variant = t.lu;
  return RB_OK;
}

int rb_solve_uneven(rb_ctx* c, int set, int B, const int* Nd, int ldu, const double* ta,
                    const double* tc, const double* tf, const double* fover, const double* u0,
                    const rb_solve_opts* opts, double* u, int* iters, int* status,
                    void* stream) {
  if (!c) return fail(RB_E_INVAL, "rb_solve_uneven: NULL context");
  Set* s = get_set(c, set);
  if (!s) return fail(RB_E_INVAL, "rb_solve_uneven: unknown set %d", set);
  if (B < 0) return fail(RB_E_INVAL, "rb_solve_uneven: B=%d", B);
  if (ldu < s->N) return fail(RB_E_INVAL, "rb_solve_uneven: ldu=%d < set N=%d", ldu, s->N);
  rb_solve_opts o = {1e-12, 10, RB_PREC_F64, 1};
  if (opts) o = *opts;
  if (int rc = check_opts("rb_solve_uneven", o)) return rc;
  if (int rc = check_lp_terms("rb_solve_uneven", s, o)) return rc;
  if (B == 0) return RB_OK;
  if (!Nd || !ta || !tc || (!tf && !fover) || !u || !iters || !status)
    return fail(RB_E_INVAL, "rb_solve_uneven: NULL array");
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc = use_device(c)) return rc;
  hipStream_t st = (hipStream_t)stream;
  const int Nm = s->N;

  // 1. per-request sizes to the host (ensure_pinned waits for any copy still reading the
  //    pinned buffer, on whichever stream it was queued)
  if (int rc = ensure_pinned(c, (size_t)3 * B + 64 * 160)) return rc;
  int* hN = c->pin;
  HIP_TRY(hipMemcpyAsync(hN, Nd, (size_t)B * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));

  // 2. same-N groups, largest N first; invalid sizes listed separately
  std::map<int, std::vector<int>, std::greater<int>> groups;
  std::vector<int> bad;
  for (int b = 0; b < B; ++b) {
    const int n = hN[b];
    if (n < 1 || n > Nm) bad.push_back(b);
    else groups[n].push_back(b);
  }
  if (o.precision == RB_PREC_F64 && !groups.empty() && groups.begin()->first > RB_MAX_N_F64)
    return fail(RB_E_UNSUPPORTED, "rb_solve_uneven: FP64 solves take N <= %d (N=%d)",
                RB_MAX_N_F64, groups.begin()->first);

  // 3. layout: staging arrays, then one state region per group (sized for region_nsplit so the
  //    autotuner can run in place)
  struct Group {
    int N;
    int64_t cnt, Bp, off;
    size_t region;
    Pack* pk;
    Tune t;
  };
  std::vector<Group> gs;
  int64_t Bs = 0;
  for (auto& kv : groups) {
    Group g;
    g.N = kv.first;
    g.cnt = (int64_t)kv.second.size();
    g.Bp = ceil_to(g.cnt, rb::kTile);
    g.off = Bs;
    Bs += g.Bp;
    gs.push_back(g);
  }
  const int nbad = (int)bad.size();
  const int fw = fover ? Nm : s->Qf;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o2 = off;
    off += (size_t)ceil_to((int64_t)bytes, 256);
    return o2;
  };
  const size_t o_ta = take(Bs * s->Q * 8), o_tc = take(Bs * s->Qc * 8), o_f = take(Bs * fw * 8);
  const size_t o_u0 = take(u0 ? Bs * Nm * 8 : 8), o_u = take(Bs * Nm * 8);
  const size_t o_it = take(Bs * 4), o_st = take(Bs * 4), o_perm = take((Bs + nbad) * 4);
  for (auto& g : gs)
    g.region = take(solve_bytes(s, g.N, g.Bp, region_nsplit(g.Bp, g.N), o.precision));
  Workspace* w;
  if (int rc = workspace(c, stream, off, &w)) return rc;
  char* base = (char*)w->buf.p;
  rb::UnevenIo io{};
  io.Bs = Bs; io.nbad = nbad; io.perm = (const int*)(base + o_perm);
  io.Q = s->Q; io.Qc = s->Qc; io.Qf = s->Qf; io.Nm = Nm; io.ldu = ldu;
  io.ta = ta; io.tc = tc; io.tf = tf; io.fover = fover; io.u0 = u0;
  io.ta_s = (double*)(base + o_ta); io.tc_s = (double*)(base + o_tc);
  io.f_s = (double*)(base + o_f); io.u0_s = (double*)(base + o_u0);
  io.u_s = (double*)(base + o_u); io.it_s = (int*)(base + o_it); io.st_s = (int*)(base + o_st);
  io.u = u; io.iters = iters; io.status = status;

  // 4. permutation to the device, gather into staging
  int* hp = c->pin + B;
  {
    int64_t r = 0;
    for (size_t i = 0; i < gs.size(); ++i) {
      const auto& src = groups[gs[i].N];
      for (int64_t k = 0; k < gs[i].Bp; ++k) hp[r++] = k < gs[i].cnt ? src[k] : -1;
    }
    for (int b : bad) hp[r++] = b;
  }
  HIP_TRY(hipMemcpyAsync(base + o_perm, hp, (size_t)(Bs + nbad) * sizeof(int),
                         hipMemcpyHostToDevice, st));
  if (int rc = pin_release(c, st)) return rc;
  if (Bs > 0)
    hipLaunchKernelGGL(rb::uneven_gather_kernel, dim3(launch_grid(Bs * Nm)), dim3(256), 0, st, io);
  HIP_TRY(hipGetLastError());

  // 5. operands and tile shapes (outside any capture: packing and tuning synchronise)
  auto args_of = [&](Group& g, int nsplit) {
    const int64_t r0 = g.off;
    return make_args(s, g.pk, g.N, (int)g.Bp, Nm, o, io.ta_s + r0 * s->Q, io.tc_s + r0 * s->Qc,
                     fover ? nullptr : io.f_s + r0 * s->Qf, fover ? io.f_s + r0 * Nm : nullptr,
                     u0 ? io.u0_s + r0 * Nm : nullptr, io.u_s + r0 * Nm, io.it_s + r0,
                     io.st_s + r0, base + g.region, nsplit);
  };
  for (auto& g : gs) {
    if (int rc = solve_pack_f64(c, s, g.N, &g.pk)) return rc;
    if (o.precision != RB_PREC_F64) {
      Pack* pl;
      if (int rc = solve_pack_lp(c, s, g.N, o.precision, &pl)) return rc;
    }
    const auto key = std::make_tuple(set, g.N, o.precision, batch_class(g.Bp));
    if (c->autotune && !c->tune.count(key)) {
      if (int rc = autotune_batch(c, s, set, args_of(g, region_nsplit(g.Bp, g.N)), o, base + g.region, st,
                                  &g.t))
        return rc;
    }
    g.t = tune_for(c, set, g.N, o.precision, g.Bp);
    // a shape tuned on another batch of the same size class may ask for more partial-sum
    // slots than this group's region holds
    g.t.nsplit = std::min(g.t.nsplit, region_nsplit(g.Bp, g.N));
  }

  // 6. the group chains: replayed from a captured graph when this shape has been seen before
  std::vector<int64_t> key = {set, o.precision, o.max_iter, o.refine_steps,
                              (int64_t)(uintptr_t)base, Bs, fover ? 1 : 0, u0 ? 1 : 0};
  int64_t tolbits;
  std::memcpy(&tolbits, &o.tol, 8);
  key.push_back(tolbits);
  for (auto& g : gs) {
    key.push_back(g.N);
    key.push_back(g.Bp);
    key.push_back(g.t.nsplit);
    key.push_back(g.t.lu);
  }
  auto run_group = [&](Group& g, hipStream_t gst) {
    return enqueue_solve(c, s, args_of(g, g.t.nsplit), o, g.t, base + g.region, gst);
  };
  GraphEntry* hit = nullptr;
  for (auto& e : c->graphs)
    if (c->uneven_graphs && e.key == key) hit = &e;
  const bool seen = c->uneven_graphs &&
                    std::find(c->seen.begin(), c->seen.end(), key) != c->seen.end();
  if (!hit && seen && !gs.empty()) {
    if (int rc = ensure_streams(c, kBranches)) return rc;
    const bool timing = c->timing;
    c->timing = false;                       // no event records inside the graph
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins;
    hipGraph_t graph = nullptr;
    int rc = RB_OK;
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(fork, c->cap_stream) != hipSuccess)
      rc = fail(RB_E_DEVICE, "rb_solve_uneven: capture fork failed");
    const int nb = std::min<int>(kBranches, (int)gs.size());
    for (int i = 0; i < nb && rc == RB_OK; ++i)
      if (hipStreamWaitEvent(c->branches[i], fork, 0) != hipSuccess)
        rc = fail(RB_E_DEVICE, "rb_solve_uneven: capture fork failed");
    for (size_t i = 0; i < gs.size() && rc == RB_OK; ++i) rc = run_group(gs[i], c->branches[i % nb]);
    for (int i = 0; i < nb && rc == RB_OK; ++i) {
      hipEvent_t j = nullptr;
      if (hipEventCreateWithFlags(&j, hipEventDisableTiming) != hipSuccess ||
          hipEventRecord(j, c->branches[i]) != hipSuccess ||
          hipStreamWaitEvent(c->cap_stream, j, 0) != hipSuccess)
        rc = fail(RB_E_DEVICE, "rb_solve_uneven: capture join failed");
      if (j) joins.push_back(j);
    }
    const hipError_t ec = hipStreamEndCapture(c->cap_stream, &graph);
    c->timing = timing;
    if (fork) (void)hipEventDestroy(fork);
    for (auto j : joins) (void)hipEventDestroy(j);
    if (rc == RB_OK && ec != hipSuccess)
      rc = fail(RB_E_DEVICE, "rb_solve_uneven: capture failed: %s", hipGetErrorString(ec));
    hipGraphExec_t exec = nullptr;
    if (rc == RB_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
      rc = fail(RB_E_DEVICE, "rb_solve_uneven: graph instantiation failed");
    if (rc != RB_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (c->graphs.size() >= kGraphCache) {
      auto lru = std::min_element(c->graphs.begin(), c->graphs.end(),
                                  [](const GraphEntry& x, const GraphEntry& y) { return x.last < y.last; });
      (void)hipGraphExecDestroy(lru->exec);
      (void)hipGraphDestroy(lru->graph);
      c->graphs.erase(lru);
    }
    GraphEntry e;
    e.key = key;
    e.graph = graph;
    e.exec = exec;
    c->graphs.push_back(e);
    hit = &c->graphs.back();
  }
  if (hit) {
    hit->last = ++c->tick;
    HIP_TRY(hipGraphLaunch(hit->exec, st));
  } else {
    for (auto& g : gs)
      if (int rc = run_group(g, st)) return rc;
    if (!seen) {
      if (c->seen.size() >= 64) c->seen.erase(c->seen.begin());
      c->seen.push_back(key);
    }
  }

  // 7. results back to the caller's order
  hipLaunchKernelGGL(rb::uneven_scatter_kernel, dim3(launch_grid((Bs + nbad) * ldu)), dim3(256),
                     0, st, io);
  HIP_TRY(hipGetLastError());
  return RB_OK;
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
  Workspace* w;
  if (int rc = workspace(c, stream, pressure_bytes(B, N, Np), &w)) return rc;
  return enqueue_pressure(c, s, B, N, Np, ldu, ldp, ta, tc, tf, tb, u, p, status,
                          (char*)w->buf.p, (hipStream_t)stream);
}

int rb_recover_pressure_uneven(rb_ctx* c, int set, int B, const int* Nd, int Np, int ldu,
                               int ldp, const double* ta, const double* tc, const double* tf,
                               const double* tb, const double* u, double* p, int* status,
                               void* stream) {
  if (!c) return fail(RB_E_INVAL, "rb_recover_pressure_uneven: NULL context");
  Set* s = get_set(c, set);
  if (!s) return fail(RB_E_INVAL, "rb_recover_pressure_uneven: unknown set %d", set);
  if (s->Np == 0)
    return fail(RB_E_INVAL, "rb_recover_pressure_uneven: set %d has no pressure data", set);
  if (B < 0) return fail(RB_E_INVAL, "rb_recover_pressure_uneven: B=%d", B);
  if (Np < 1 || Np > s->Np || ldu < s->N || ldp < Np)
    return fail(RB_E_INVAL, "rb_recover_pressure_uneven: Np=%d ldu=%d ldp=%d out of range", Np,
                ldu, ldp);
  if (B == 0) return RB_OK;
  if (!Nd || !ta || !tc || !tf || !tb || !u || !p || !status)
    return fail(RB_E_INVAL, "rb_recover_pressure_uneven: NULL array");
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc = use_device(c)) return rc;
  hipStream_t st = (hipStream_t)stream;
  const int Nm = s->N;
  if (int rc = ensure_pinned(c, (size_t)3 * B + 64 * 160)) return rc;
  int* hN = c->pin;
  HIP_TRY(hipMemcpyAsync(hN, Nd, (size_t)B * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  std::map<int, std::vector<int>, std::greater<int>> groups;
  std::vector<int> bad;
  for (int b = 0; b < B; ++b) {
    const int n = hN[b];
    if (n < 1 || n > Nm) bad.push_back(b);
    else groups[n].push_back(b);
  }
  struct Group { int N; int64_t cnt, Bp, off; size_t part; };
  std::vector<Group> gs;
  int64_t Bs = 0;
  for (auto& kv : groups) {
    Group g;
    g.N = kv.first;
    g.cnt = (int64_t)kv.second.size();
    g.Bp = ceil_to(g.cnt, rb::kTile);
    g.off = Bs;
    Bs += g.Bp;
    gs.push_back(g);
  }
  const int nbad = (int)bad.size();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o2 = off;
    off += (size_t)ceil_to((int64_t)bytes, 256);
    return o2;
  };
  const size_t o_ta = take(Bs * s->Q * 8), o_tc = take(Bs * s->Qc * 8), o_tf = take(Bs * s->Qf * 8);
  const size_t o_tb = take(Bs * s->Qb * 8), o_u = take(Bs * Nm * 8), o_p = take(Bs * Np * 8);
  const size_t o_st = take(Bs * 4), o_dummy = take((size_t)B * 4), o_perm = take((Bs + nbad) * 4);
  for (auto& g : gs) g.part = take(pressure_bytes((int)g.cnt, g.N, Np));
  Workspace* w;
  if (int rc = workspace(c, stream, off, &w)) return rc;
  char* base = (char*)w->buf.p;
  int* hp = c->pin + B;
  {
    int64_t r = 0;
    for (auto& g : gs) {
      const auto& src = groups[g.N];
      for (int64_t k = 0; k < g.Bp; ++k) hp[r++] = k < g.cnt ? src[k] : -1;
    }
    for (int b : bad) hp[r++] = b;
  }
  HIP_TRY(hipMemcpyAsync(base + o_perm, hp, (size_t)(Bs + nbad) * sizeof(int),
                         hipMemcpyHostToDevice, st));
  if (int rc = pin_release(c, st)) return rc;
  // gather theta and u (into the u0 staging slot) in group order
  rb::UnevenIo io{};
  io.Bs = Bs; io.nbad = nbad; io.perm = (const int*)(base + o_perm);
  io.Q = s->Q; io.Qc = s->Qc; io.Qf = s->Qf; io.Nm = Nm; io.ldu = ldu;
  io.ta = ta; io.tc = tc; io.tf = tf; io.fover = nullptr; io.u0 = u;
  io.ta_s = (double*)(base + o_ta); io.tc_s = (double*)(base + o_tc);
  io.f_s = (double*)(base + o_tf); io.u0_s = (double*)(base + o_u);
  io.tb = tb; io.tb_s = (double*)(base + o_tb); io.Qb = s->Qb;
  if (Bs > 0)
    hipLaunchKernelGGL(rb::uneven_gather_kernel, dim3(launch_grid(Bs * Nm)), dim3(256), 0, st, io);
  HIP_TRY(hipGetLastError());
  double* p_s = (double*)(base + o_p);
  int* st_s = (int*)(base + o_st);
  for (auto& g : gs) {
    const int64_t r0 = g.off;
    if (int rc = enqueue_pressure(c, s, (int)g.cnt, g.N, Np, Nm, Np, io.ta_s + r0 * s->Q,
                                  io.tc_s + r0 * s->Qc, io.f_s + r0 * s->Qf,
                                  io.tb_s + r0 * s->Qb, io.u0_s + r0 * Nm, p_s + r0 * Np,
                                  st_s + r0, base + g.part, st))
      return rc;
  }
  // scatter p and the statuses back (rows of length Np, caller stride ldp)
  rb::UnevenIo so{};
  so.Bs = Bs; so.nbad = nbad; so.perm = io.perm;
  so.Nm = Np; so.ldu = ldp;
  so.u_s = p_s; so.it_s = st_s; so.st_s = st_s;
  so.u = p; so.iters = (int*)(base + o_dummy); so.status = status;
  hipLaunchKernelGGL(rb::uneven_scatter_kernel, dim3(launch_grid((Bs + nbad) * ldp)), dim3(256),
                     0, st, so);
  HIP_TRY(hipGetLastError());
  return RB_OK;
}

int rb_reconstruct_pressure(rb_ctx* c, int B, int N, int Np, const double* Pc, int ldpc,
                            const double* u, int ldu, double* p, int ldp, void* stream) {
  if (!c) return fail(RB_E_INVAL, "rb_reconstruct_pressure: NULL context");
  if (B < 0 || N < 1 || N > RB_MAX_N || Np < 1 || Np > RB_MAX_NP)
    return fail(RB_E_INVAL, "rb_reconstruct_pressure: B=%d N=%d Np=%d out of range", B, N, Np);
  if (ldpc < N || ldu < N || ldp < Np)
    return fail(RB_E_INVAL, "rb_reconstruct_pressure: ldpc=%d ldu=%d ldp=%d too small", ldpc,
                ldu, ldp);
  if (B == 0) return RB_OK;
  if (!Pc || !u || !p) return fail(RB_E_INVAL, "rb_reconstruct_pressure: NULL array");
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc = use_device(c)) return rc;
  const size_t lds = (size_t)N * Np * sizeof(double);
  if (lds > 64 * 1024)
    HIP_TRY(hipFuncSetAttribute((const void*)rb::reconstruct_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const int64_t total = (int64_t)B * ldp;
  const int grid = (int)std::min<int64_t>(2048, (total + 255) / 256);
  LaunchTimer t(c, FAM_RECONSTRUCT, (hipStream_t)stream);
  hipLaunchKernelGGL(rb::reconstruct_kernel, dim3(grid), dim3(256), lds, (hipStream_t)stream, Pc,
                     ldpc, N, Np, B, u, ldu, p, ldp);
  HIP_TRY(hipGetLastError());
  return RB_OK;
}

int rb_assemble_convection(rb_ctx* c, int N, int R, int X, int Qc, const double* phiT,
                           const double* dphiT, const double* testT, const double* M, double w,
                           double* out, void* stream) {
  if (!c) return fail(RB_E_INVAL, "rb_assemble_convection: NULL context");
  if (N < 1 || N > RB_MAX_N || R < 1 || R > RB_MAX_N || X < 1 || Qc < 1 || Qc > RB_MAX_QC)
    return fail(RB_E_INVAL, "rb_assemble_convection: N=%d R=%d X=%d Qc=%d out of range", N, R,
                X, Qc);
  if (!phiT || !dphiT || !testT || !M || !out)
    return fail(RB_E_INVAL, "rb_assemble_convection: NULL array");
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc = use_device(c)) return rc;
  hipStream_t st = (hipStream_t)stream;
  const int64_t wgs = (int64_t)((R + 63) / 64) * ((N + rb::kAsmWaves - 1) / rb::kAsmWaves) *
                      ((N + 15) / 16);
  // split the quadrature points until about 4096 wavefronts run (at most 16 splits, and at
  // least 64 points per split)
  int nsx = (int)std::min<int64_t>(16, std::max<int64_t>(1, (4096 + 4 * wgs - 1) / (4 * wgs)));
  nsx = std::max(1, std::min(nsx, X / 64));
  const size_t part_bytes = (size_t)nsx * 4 * R * N * N * sizeof(double);
  Workspace* ws;
  if (int rc = workspace(c, stream, part_bytes + 4 * Qc * sizeof(double) + 256, &ws)) return rc;
  double* part = (double*)ws->buf.p;
  double* Md = (double*)((char*)ws->buf.p + ceil_to((int64_t)part_bytes, 256));
  HIP_TRY(hipMemcpyAsync(Md, M, 4 * Qc * sizeof(double), hipMemcpyHostToDevice, st));
  rb::AssembleArgs g{N, R, X, nsx, phiT, dphiT, testT, part};
  hipLaunchKernelGGL(rb::assemble_conv_kernel, dim3((unsigned)(wgs * nsx)),
                     dim3(rb::kWave * rb::kAsmWaves), 0, st, g);
  HIP_TRY(hipGetLastError());
  const int64_t per = (int64_t)R * N * N;
  hipLaunchKernelGGL(rb::assemble_combine_kernel, dim3(launch_grid(per)), dim3(256), 0, st,
                     (const double*)part, nsx, R, N, Qc, (const double*)Md, w, out);
  HIP_TRY(hipGetLastError());
  // the host copy of M has been read; wait so that the caller may release it
  HIP_TRY(hipStreamSynchronize(st));
  return RB_OK;
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

// ------------------------------------------------------------------ serving ----------
namespace {

using Clock = std::chrono::steady_clock;

struct Pending {
  long long ticket, tag;
  int N;
  double alpha, re;
  Clock::time_point t_submit;
};

// Waiting requests, one FIFO per size class (key: the class size) plus the requests with an
// invalid N; the oldest waiting request is the smallest ticket among the class fronts, so
// taking a class costs the batch it takes, whatever the length of the queue.
struct WaitQueue {
  std::map<int, std::deque<Pending>> cls;
  std::deque<Pending> bad;
  size_t n = 0;                       // requests in cls
  bool empty() const { return n == 0 && bad.empty(); }
};

// Latency quantiles in bounded memory: log-spaced bins of ratio 1.01 from 1 us to 1000 s
// (2083 bins), so a quantile is known to within 0.5 %, whatever the number of requests.
struct LatHist {
  static constexpr double kLo = 1e-3, kRatio = 1.01;   // ms
  std::vector<uint64_t> bins = std::vector<uint64_t>(2084, 0);
  uint64_t n = 0;
  double maxv = 0.0;
  void add(double ms) {
    const double x = std::max(ms, kLo);
    const size_t b = std::min(bins.size() - 1, (size_t)(std::log(x / kLo) / std::log(kRatio)));
    ++bins[b];
    ++n;
    maxv = std::max(maxv, ms);
  }
  double quantile(double f) const {
    if (n == 0) return 0.0;
    const uint64_t want = std::min<uint64_t>(n - 1, (uint64_t)(f * (double)(n - 1) + 0.5));
    uint64_t seen = 0;
    for (size_t b = 0; b < bins.size(); ++b) {
      seen += bins[b];
      if (seen > want) return std::min(maxv, kLo * std::pow(kRatio, (double)b + 0.5));
    }
    return maxv;
  }
};

// One lane: a stream, its device buffers for max_batch requests and pinned host mirrors. The
// worker admits one size class per batch, so a lane's batch runs in order on its one stream
// (lanes map one to one onto the device's hardware queues: extra streams per lane would only
// queue behind other lanes' long kernels).
struct Lane {
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  Clock::time_point t_launch;         // when the batch in flight was launched
  size_t need = 0;                    // workspace estimate of the batch in flight
  std::vector<Pending> batch;         // in the order of the device rows (grouped by N)
  DevBuf d_mu, d_ta, d_tc, d_tf, d_tb, d_u, d_p, d_int, d_n;
  double* h_mu = nullptr;             // pinned [cap][2]
  int* h_n = nullptr;                 // pinned [cap]: basis size of each row
  double* h_u = nullptr;              // pinned [cap][Nm]
  double* h_p = nullptr;              // pinned [cap][Np]
  int* h_int = nullptr;               // pinned [3][cap]: iters, status, pstatus
};

}  // namespace

struct rb_server {
  rb_ctx* c = nullptr;
  int set = 0;
  Set* s = nullptr;
  rb_server_opts o{};
  int cap = 0;
  std::vector<Lane> lanes;
  std::thread worker;
  std::mutex qm;                      // queue, results, stats
  std::condition_variable qcv;
  WaitQueue queue;
  std::deque<rb_result> results;
  bool stopping = false;
  long long next_ticket = 1, submitted = 0, completed = 0, batches = 0;
  LatHist lat, wait;                  // latency and queue-wait histograms
  Clock::time_point t0;
  double first_submit_s = -1.0, last_done_s = 0.0;
  size_t inflight = 0, inflight_peak = 0;
  std::string error;
};

namespace {

// Group size of a served request of basis size n: n rounded up to a multiple of 16 (at most
// the set's N). A request is solved as the leading n x n block of its group's system (the
// remaining unknowns held at zero by identity rows), so a batch with many distinct sizes runs
// a handful of group chains; the group depends on n only, so a request's result does not
// depend on the rest of its batch.
int serve_group(int n, int Nm) { return (int)std::min<int64_t>(Nm, ceil_to(n, 16)); }

// Tile shape of a served group of size N: the row split a single 64-request tile gets by
// default, whatever the batch size and whatever the tuning table holds. The partial sums of
// A(mu) u (and of the pressure right-hand side) are then added in the same order for a
// request alone and in any mix, so its result is the same bit for bit.
Tune serve_tune(int N, int lu) {
  Tune t;
  t.nsplit = default_nsplit(rb::kTile, N * N);
  t.lu = lu;
  return t;
}
int serve_press_nsplit(int N, int Np) { return default_nsplit(rb::kTile, Np * N); }

// Workspace of one batch: per N group the Newton state and, with pressure, the pressure
// partial sums.
size_t batch_bytes(rb_server* v, const std::vector<std::pair<int, int>>& groups) {
  size_t b = 0;
  for (auto& g : groups) {
    const int N = g.first, Np = v->s->Np;
    const int64_t Bp = ceil_to(g.second, rb::kTile);
    b += solve_bytes(v->s, N, Bp, serve_tune(N, v->c->lu).nsplit, v->o.precision);
    if (v->o.pressure)
      b += (size_t)ceil_to((int64_t)pressure_bytes(g.second, N, Np, serve_press_nsplit(N, Np)),
                           256);
  }
  return b;
}

// Launch one batch on a lane (caller holds the context lock). Rows are grouped by N, largest
// first; each group runs as a same-N batch on the lane's stream.
int launch_batch(rb_server* v, Lane& L) {
  rb_ctx* c = v->c;
  Set* s = v->s;
  const int Nm = s->N, Np = s->Np, B = (int)L.batch.size();
  for (int i = 0; i < B; ++i) {
    L.h_mu[2 * i] = L.batch[i].alpha;
    L.h_mu[2 * i + 1] = L.batch[i].re;
    L.h_n[i] = L.batch[i].N;
  }
  HIP_TRY(hipMemcpyAsync(L.d_mu.p, L.h_mu, (size_t)B * 2 * sizeof(double), hipMemcpyHostToDevice,
                         L.st));
  HIP_TRY(hipMemcpyAsync(L.d_n.p, L.h_n, (size_t)B * sizeof(int), hipMemcpyHostToDevice, L.st));
  const int Qb = Np > 0 ? s->Qb : 1;
  double* ta = (double*)L.d_ta.p;
  double* tc = (double*)L.d_tc.p;
  double* tf = (double*)L.d_tf.p;
  double* tb = (double*)L.d_tb.p;
  hipLaunchKernelGGL(rb::theta_kernel, dim3((B + 255) / 256), dim3(256), 0, L.st,
                     (const double*)L.d_mu.p, B, s->Q, s->Qc, s->Qf, Qb, ta, tc, tf,
                     Np > 0 ? tb : nullptr);
  std::vector<std::pair<int, int>> groups;   // (group size, count), rows contiguous
  for (int i = 0; i < B;) {
    const int gN = serve_group(L.batch[i].N, Nm);
    int j = i;
    while (j < B && serve_group(L.batch[j].N, Nm) == gN) ++j;
    groups.push_back({gN, j - i});
    i = j;
  }
  Workspace* w;
  if (int rc = workspace(c, L.st, batch_bytes(v, groups), &w)) return rc;
  char* base = (char*)w->buf.p;
  double* u = (double*)L.d_u.p;
  double* p = (double*)L.d_p.p;
  int* it = (int*)L.d_int.p;
  int* stt = it + v->cap;
  int* pst = it + 2 * v->cap;
  rb_solve_opts o = {v->o.tol, v->o.max_iter, v->o.precision, v->o.refine_steps};
  // one group per size class (a batch holds one class), in order on the lane's stream
  int r0 = 0;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const auto& g = groups[gi];
    hipStream_t gst = L.st;
    const int N = g.first, n = g.second;
    const int64_t Bp = ceil_to(n, rb::kTile);
    Pack* pk;
    if (int rc = solve_pack_f64(c, s, N, &pk)) return rc;
    const Tune t = serve_tune(N, c->lu);
    rb::NewtonF64Args a =
        make_args(s, pk, N, n, Nm, o, ta + (int64_t)r0 * s->Q, tc + (int64_t)r0 * s->Qc,
                  tf + (int64_t)r0 * s->Qf, nullptr, nullptr, u + (int64_t)r0 * Nm, it + r0,
                  stt + r0, base, t.nsplit, (const int*)L.d_n.p + r0);
    if (int rc = enqueue_solve(c, s, a, o, t, base, gst)) return rc;
    base += solve_bytes(s, N, Bp, t.nsplit, o.precision);
    if (v->o.pressure) {
      if (int rc = enqueue_pressure(c, s, n, N, Np, Nm, Np, ta + (int64_t)r0 * s->Q,
                                    tc + (int64_t)r0 * s->Qc, tf + (int64_t)r0 * s->Qf,
                                    tb + (int64_t)r0 * s->Qb, u + (int64_t)r0 * Nm,
                                    p + (int64_t)r0 * Np, pst + r0, base, gst,
                                    serve_press_nsplit(N, Np)))
        return rc;
      base += (size_t)ceil_to((int64_t)pressure_bytes(n, N, Np, serve_press_nsplit(N, Np)), 256);
    }
    r0 += n;
  }
  HIP_TRY(hipMemcpyAsync(L.h_u, u, (size_t)B * Nm * sizeof(double), hipMemcpyDeviceToHost, L.st));
  HIP_TRY(hipMemcpyAsync(L.h_int, it, (size_t)3 * v->cap * sizeof(int), hipMemcpyDeviceToHost, L.st));
  if (v->o.pressure)
    HIP_TRY(hipMemcpyAsync(L.h_p, p, (size_t)B * Np * sizeof(double), hipMemcpyDeviceToHost, L.st));
  HIP_TRY(hipEventRecord(L.done, L.st));
  return RB_OK;
}

// Results of a finished lane into the result queue (caller holds v->qm).
void harvest(rb_server* v, Lane& L, bool failed) {
  const int Nm = v->s->N, Np = v->s->Np;
  const auto now = Clock::now();
  for (size_t i = 0; i < L.batch.size(); ++i) {
    const Pending& q = L.batch[i];
    rb_result r;
    std::memset(&r, 0, sizeof r);
    r.ticket = q.ticket;
    r.tag = q.tag;
    r.N = q.N;
    if (failed) {
      r.status = RB_ST_FAILED;
      r.pstatus = RB_ST_FAILED;
    } else {
      r.iters = L.h_int[i];
      r.status = L.h_int[v->cap + i];
      r.pstatus = v->o.pressure ? L.h_int[2 * v->cap + i] : 0;
      for (int k = 0; k < q.N; ++k) r.u[k] = L.h_u[(size_t)i * Nm + k];
      if (v->o.pressure)
        for (int k = 0; k < Np; ++k) r.p[k] = L.h_p[(size_t)i * Np + k];
    }
    r.latency_ms = std::chrono::duration<double, std::milli>(now - q.t_submit).count();
    r.queue_ms = std::chrono::duration<double, std::milli>(L.t_launch - q.t_submit).count();
    v->lat.add(r.latency_ms);
    v->wait.add(r.queue_ms);
    v->results.push_back(r);
  }
  v->completed += (long long)L.batch.size();
  v->last_done_s = std::chrono::duration<double>(now - v->t0).count();
  v->inflight -= L.need;
  L.batch.clear();
  L.busy = false;
}

void bad_request(rb_server* v, const Pending& q) {
  rb_result r;
  std::memset(&r, 0, sizeof r);
  r.ticket = q.ticket;
  r.tag = q.tag;
  r.N = q.N;
  r.status = RB_ST_BADN;
  r.pstatus = RB_ST_BADN;
  r.latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - q.t_submit).count();
  r.queue_ms = r.latency_ms;
  v->lat.add(r.latency_ms);
  v->wait.add(r.queue_ms);
  v->results.push_back(r);
  ++v->completed;
}

void serve(rb_server* v) {
  (void)hipSetDevice(v->c->device);
  std::unique_lock<std::mutex> lk(v->qm);
  for (;;) {
    bool progress = false;
    // 1. retire finished lanes
    for (auto& L : v->lanes) {
      if (!L.busy) continue;
      const hipError_t q = hipEventQuery(L.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) v->error = hipGetErrorString(q);
      harvest(v, L, q != hipSuccess);
      progress = true;
    }
    // 2. admit: a free lane takes the size class of the oldest waiting request, every
    //    queued request of that class (in arrival order) up to max_batch and the HBM budget;
    //    the other classes keep their place for the next free lane
    for (auto& L : v->lanes) {
      if (L.busy) continue;
      const int Nm = v->s->N;
      WaitQueue& wq = v->queue;
      for (const Pending& q : wq.bad) bad_request(v, q);
      progress = progress || !wq.bad.empty();
      wq.bad.clear();
      if (wq.n == 0) continue;
      std::deque<Pending>* oldest = nullptr;
      for (auto& kv : wq.cls)
        if (!kv.second.empty() && (!oldest || kv.second.front().ticket < oldest->front().ticket))
          oldest = &kv.second;
      std::vector<Pending> take;
      while (!oldest->empty() && (int)take.size() < v->cap) {
        take.push_back(oldest->front());
        oldest->pop_front();
      }
      wq.n -= take.size();
      auto groups_of = [Nm](const std::vector<Pending>& t, size_t n) {
        std::vector<std::pair<int, int>> g;
        for (size_t i = 0; i < n; ++i) {
          const int gN = serve_group(t[i].N, Nm);
          if (g.empty() || g.back().first != gN) g.push_back({gN, 0});
          ++g.back().second;
        }
        return g;
      };
      size_t n = take.size();
      size_t need = batch_bytes(v, groups_of(take, n));
      const size_t budget = v->o.hbm_budget_bytes;
      while (budget && n > 1 && v->inflight + need > budget) {   // cut to what fits
        n = n / 2;
        need = batch_bytes(v, groups_of(take, n));
      }
      if (budget && v->inflight + need > budget && v->inflight > 0) n = 0;   // wait for room
      for (size_t i = take.size(); i-- > n;) oldest->push_front(take[i]);
      wq.n += take.size() - n;
      if (n == 0) continue;
      take.resize(n);
      L.batch = std::move(take);
      L.need = need;
      L.busy = true;
      v->inflight += need;
      v->inflight_peak = std::max(v->inflight_peak, v->inflight);
      ++v->batches;
      L.t_launch = Clock::now();
      // Launch without the queue lock, so that submitters are not held up for the host time
      // of the launches; only this thread touches the lanes.
      lk.unlock();
      int rc;
      {
        std::lock_guard<std::mutex> ck(v->c->mu);   // workspaces, packed operands, launches
        rc = launch_batch(v, L);
        if (rc != RB_OK) {
          (void)hipStreamSynchronize(L.st);
        }
      }
      const std::string err = rc != RB_OK ? g_err : std::string();
      lk.lock();
      if (rc != RB_OK) {
        v->error = err;
        harvest(v, L, true);
      }
      progress = true;
    }
    bool idle = v->queue.empty();
    for (auto& L : v->lanes) idle = idle && !L.busy;
    if (v->stopping && idle) break;
    if (!progress) {
      bool any_busy = false;
      for (auto& L : v->lanes) any_busy = any_busy || L.busy;
      // lanes in flight: poll again shortly; nothing to do: sleep until a submission
      if (any_busy) v->qcv.wait_for(lk, std::chrono::microseconds(20));
      else v->qcv.wait(lk, [&] { return v->stopping || !v->queue.empty(); });
    }
  }
}

void free_lanes(rb_server* v) {
  for (auto& L : v->lanes) {
    for (DevBuf* b : {&L.d_mu, &L.d_ta, &L.d_tc, &L.d_tf, &L.d_tb, &L.d_u, &L.d_p, &L.d_int, &L.d_n})
      dev_free(v->c, *b);
    for (void* h : {(void*)L.h_mu, (void*)L.h_u, (void*)L.h_p, (void*)L.h_int, (void*)L.h_n})
      if (h) (void)hipHostFree(h);
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.st) {
      auto it = v->c->ws.find((void*)L.st);
      if (it != v->c->ws.end()) {
        dev_free(v->c, it->second.buf);
        v->c->ws.erase(it);
      }
      (void)hipStreamDestroy(L.st);
    }
  }
  v->lanes.clear();
}

}  // namespace

extern "C" {

int rb_server_start(rb_ctx* c, int set, const rb_server_opts* opts, rb_server** out) {
  if (!c || !opts || !out) return fail(RB_E_INVAL, "rb_server_start: NULL argument");
  *out = nullptr;
  Set* s = get_set(c, set);
  if (!s) return fail(RB_E_INVAL, "rb_server_start: unknown set %d", set);
  const rb_server_opts& o = *opts;
  rb_solve_opts so = {o.tol, o.max_iter, o.precision, o.refine_steps};
  if (int rc = check_opts("rb_server_start", so)) return rc;
  if (int rc = check_lp_terms("rb_server_start", s, so)) return rc;
  if (o.precision == RB_PREC_F64 && s->N > RB_MAX_N_F64)
    return fail(RB_E_UNSUPPORTED, "rb_server_start: FP64 serving takes set N <= %d",
                RB_MAX_N_F64);
  if (o.max_batch < 1 || o.max_batch > 65536 || o.lanes < 1 || o.lanes > 16)
    return fail(RB_E_INVAL, "rb_server_start: max_batch=%d lanes=%d", o.max_batch, o.lanes);
  if (o.pressure && s->Np == 0)
    return fail(RB_E_INVAL, "rb_server_start: set %d has no pressure data", set);
  std::unique_ptr<rb_server> v(new rb_server);
  v->c = c;
  v->set = set;
  v->s = s;
  v->o = o;
  v->cap = o.max_batch;
  v->t0 = Clock::now();
  {
    std::lock_guard<std::mutex> ck(c->mu);
    if (int rc = use_device(c)) return rc;
    const size_t cap = v->cap, Nm = s->N, Np = std::max(1, s->Np);
    v->lanes.resize(o.lanes);
    for (auto& L : v->lanes) {
      int rc = RB_OK;
      if (hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess)
        rc = fail(RB_E_DEVICE, "rb_server_start: stream/event creation failed");
      if (!rc) rc = dev_alloc(c, L.d_mu, cap * 2 * 8);
      if (!rc) rc = dev_alloc(c, L.d_ta, cap * s->Q * 8);
      if (!rc) rc = dev_alloc(c, L.d_tc, cap * s->Qc * 8);
      if (!rc) rc = dev_alloc(c, L.d_tf, cap * s->Qf * 8);
      if (!rc) rc = dev_alloc(c, L.d_tb, cap * std::max(1, s->Qb) * 8);
      if (!rc) rc = dev_alloc(c, L.d_u, cap * Nm * 8);
      if (!rc) rc = dev_alloc(c, L.d_p, cap * Np * 8);
      if (!rc) rc = dev_alloc(c, L.d_int, cap * 3 * 4);
      if (!rc) rc = dev_alloc(c, L.d_n, cap * 4);
      if (!rc && (hipHostMalloc((void**)&L.h_mu, cap * 2 * 8, hipHostMallocDefault) != hipSuccess ||
                  hipHostMalloc((void**)&L.h_u, cap * Nm * 8, hipHostMallocDefault) != hipSuccess ||
                  hipHostMalloc((void**)&L.h_p, cap * Np * 8, hipHostMallocDefault) != hipSuccess ||
                  hipHostMalloc((void**)&L.h_int, cap * 3 * 4, hipHostMallocDefault) != hipSuccess ||
                  hipHostMalloc((void**)&L.h_n, cap * 4, hipHostMallocDefault) != hipSuccess))
        rc = fail(RB_E_NOMEM, "rb_server_start: pinned host buffers");
      if (rc) {
        free_lanes(v.get());
        return rc;
      }
    }
    // packed operands of every basis size are built on first use; build the full one now,
    // and size each lane's workspace for a full batch at the largest basis size, so that
    // batches do not wait for a workspace to grow
    Pack* pk;
    if (int rc = solve_pack_f64(c, s, s->N, &pk)) {
      free_lanes(v.get());
      return rc;
    }
    const size_t ws = batch_bytes(v.get(), {{s->N, v->cap}});
    if (!o.hbm_budget_bytes || ws <= o.hbm_budget_bytes) {
      for (auto& L : v->lanes) {
        Workspace* w;
        if (int rc = workspace(c, L.st, ws, &w)) {
          free_lanes(v.get());
          return rc;
        }
      }
    }
  }
  rb_server* raw = v.release();
  raw->worker = std::thread(serve, raw);
  *out = raw;
  return RB_OK;
}

int rb_server_submit(rb_server* v, const rb_request* reqs, int n, long long* tickets) {
  if (!v || (n > 0 && !reqs) || n < 0) return fail(RB_E_INVAL, "rb_server_submit: bad argument");
  const auto now = Clock::now();
  {
    std::lock_guard<std::mutex> lk(v->qm);
    if (v->stopping) return fail(RB_E_STATE, "rb_server_submit: server is stopping");
    if (v->first_submit_s < 0 && n > 0)
      v->first_submit_s = std::chrono::duration<double>(now - v->t0).count();
    for (int i = 0; i < n; ++i) {
      Pending q;
      q.ticket = v->next_ticket++;
      q.tag = reqs[i].tag;
      q.N = reqs[i].N;
      q.alpha = reqs[i].alpha;
      q.re = reqs[i].re;
      q.t_submit = now;
      if (q.N < 1 || q.N > v->s->N) {
        v->queue.bad.push_back(q);
      } else {
        v->queue.cls[serve_group(q.N, v->s->N)].push_back(q);
        ++v->queue.n;
      }
      if (tickets) tickets[i] = q.ticket;
    }
    v->submitted += n;
  }
  v->qcv.notify_one();
  return RB_OK;
}

int rb_server_poll(rb_server* v, rb_result* out, int max, int* n_out) {
  if (!v || !n_out || (max > 0 && !out)) return fail(RB_E_INVAL, "rb_server_poll: bad argument");
  std::lock_guard<std::mutex> lk(v->qm);
  int n = 0;
  while (n < max && !v->results.empty()) {
    out[n++] = v->results.front();
    v->results.pop_front();
  }
  *n_out = n;
  return RB_OK;
}

int rb_server_stats(rb_server* v, rb_server_counters* st) {
  if (!v || !st) return fail(RB_E_INVAL, "rb_server_stats: NULL argument");
  std::lock_guard<std::mutex> lk(v->qm);
  std::memset(st, 0, sizeof *st);
  st->submitted = v->submitted;
  st->completed = v->completed;
  st->batches = v->batches;
  st->p50_ms = v->lat.quantile(0.50);
  st->p99_ms = v->lat.quantile(0.99);
  st->max_ms = v->lat.maxv;
  st->p50_queue_ms = v->wait.quantile(0.50);
  st->p99_queue_ms = v->wait.quantile(0.99);
  st->mean_batch = v->batches ? (double)(v->completed) / v->batches : 0.0;
  st->first_submit_s = v->first_submit_s;
  st->last_done_s = v->last_done_s;
  st->hbm_inflight_peak = v->inflight_peak;
  std::snprintf(st->error, sizeof st->error, "%s", v->error.c_str());
  return RB_OK;
}

int rb_server_stop(rb_server* v) {
  if (!v) return fail(RB_E_INVAL, "rb_server_stop: NULL server");
  {
    std::lock_guard<std::mutex> lk(v->qm);
    v->stopping = true;
  }
  v->qcv.notify_one();
  if (v->worker.joinable()) v->worker.join();
  {
    std::lock_guard<std::mutex> ck(v->c->mu);
    (void)hipSetDevice(v->c->device);
    for (auto& L : v->lanes) {
      if (L.st) (void)hipStreamSynchronize(L.st);
    }
    free_lanes(v);
  }
  delete v;
  return RB_OK;
}

}  // extern "C"
