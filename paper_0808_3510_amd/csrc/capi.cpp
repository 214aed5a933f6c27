// C ABI of libpatnufft (declared in include/pat.h).  Validates every argument
// before enqueueing anything and converts failures into status codes.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "launch.h"
#include "plan.h"

namespace {

thread_local std::string g_err;

pat_status set_err(pat_status s, const std::string& m) {
  g_err = m;
  return s;
}

pat_status hip_err(hipError_t e, const char* where) {
  return set_err(PAT_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

bool aligned16(const void* p) { return p && (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// The PAT_FAULT hook, read at the start of every call that touches the GPU:
//   upload    pat_plan_upload's copy fails,
//   scratch   pat_reconstruct_noalloc's scratch lookup fails,
//   launch[:k] the k-th kernel launch of the operator fails (default 1),
// each as a HIP error reported before that step runs.  Unset: no effect.
struct Faults {
  bool upload = false, scratch = false;
};
Faults arm_faults() {
  Faults f;
  int k = 0;
  const char* v = std::getenv("PAT_FAULT");
  if (v && *v) {
    if (std::strcmp(v, "upload") == 0) {
      f.upload = true;
    } else if (std::strcmp(v, "scratch") == 0) {
      f.scratch = true;
    } else if (std::strncmp(v, "launch", 6) == 0) {
      k = 1;
      if (v[6] == ':') k = std::atoi(v + 7);
    }
  }
  pat::set_launch_fault(k);
  return f;
}

// hipEvent pairs around each kernel of a transform.
class EventTimer : public pat::StageTimer {
 public:
  ~EventTimer() override {
    for (hipEvent_t e : ev_) (void)hipEventDestroy(e);
  }
  void reset() {
    names_.clear();
    used_ = 0;
  }
  void begin(const char* name, hipStream_t s) override {
    names_.push_back(name);
    (void)hipEventRecord(get(), s);
  }
  void end(hipStream_t s) override { (void)hipEventRecord(get(), s); }
  int count() const { return (int)names_.size(); }
  const char* name(int i) const { return names_[i]; }
  float ms(int i) {
    float v = 0.f;
    (void)hipEventSynchronize(ev_[2 * i + 1]);
    (void)hipEventElapsedTime(&v, ev_[2 * i], ev_[2 * i + 1]);
    return v;
  }

 private:
  hipEvent_t get() {
    if (used_ == ev_.size()) {
      hipEvent_t e;
      (void)hipEventCreate(&e);
      ev_.push_back(e);
    }
    return ev_[used_++];
  }
  std::vector<const char*> names_;
  std::vector<hipEvent_t> ev_;
  size_t used_ = 0;
};

// Records accumulate over calls until pat_plan_stage_times() reads them.
EventTimer* timer_of(pat_plan* p) {
  if (!p->timing) return nullptr;
  if (!p->timer) p->timer = new (std::nothrow) EventTimer();
  return static_cast<EventTimer*>(p->timer);
}

pat_status check_plan(const pat_plan* p) {
  if (!p) return set_err(PAT_ERR_INVALID_ARG, "plan is NULL");
  if (!p->uploaded) return set_err(PAT_ERR_WORKSPACE, "plan tables not uploaded (pat_plan_upload)");
  return PAT_OK;
}

// Bytes of a plan's detector data (nt per column) or image (nz per column).
size_t column_array_bytes(const pat_plan* p, bool image) {
  const pat::Inst& I = p->inst;
  return (size_t)I.n1 * I.n2 * (image ? I.nz : I.nt) * (pat::complex_bytes(p->prec) / 2);
}

pat_status check_size(const char* what, size_t have, size_t need, pat_status code) {
  if (have >= need) return PAT_OK;
  return set_err(code, std::string(what) + " holds " + std::to_string(have) + " bytes, the plan needs " +
                           std::to_string(need));
}

// Checks shared by the single-plan operators (workspace aside).
pat_status check_call(pat_plan* plan, pat::Op op, const void* in, size_t in_bytes, void* out, size_t out_bytes) {
  pat_status s = check_plan(plan);
  if (s != PAT_OK) return s;
  if (!aligned16(in) || !aligned16(out)) return set_err(PAT_ERR_INVALID_ARG, "input/output NULL or not 16-byte aligned");
  const bool in_image = op == pat::OP_RT || op == pat::OP_A;
  s = check_size("input array", in_bytes, column_array_bytes(plan, in_image), PAT_ERR_INVALID_ARG);
  if (s != PAT_OK) return s;
  s = check_size("output array", out_bytes, column_array_bytes(plan, !in_image), PAT_ERR_INVALID_ARG);
  if (s != PAT_OK) return s;
  if (op != pat::OP_R && plan->inst.kind != PAT_INTERP_KB)
    return set_err(PAT_ERR_UNSUPPORTED, "only the reconstruction runs with an interp other than PAT_INTERP_KB");
  if ((op == pat::OP_RT || op == pat::OP_A) && !plan->spread_ok)
    return set_err(PAT_ERR_UNSUPPORTED, "nz too large for the spreading lists of a depth line in LDS");
  return PAT_OK;
}

// Enqueues one operator of one plan; h: the host descriptor (its workspace
// offsets place the stages' arrays in ws).
pat_status enqueue(pat_plan* plan, const pat::Inst& h, pat::Op op, const void* in, void* out, void* ws, void* stream,
                   pat::StageTimer* tm) {
  const pat::Inst* d = reinterpret_cast<const pat::Inst*>(static_cast<unsigned char*>(plan->table_dev) + plan->off_desc);
  const pat::Inst* dd[1] = {d};
  const void* ins[1] = {in};
  void* outs[1] = {out};
  void* wss[1] = {ws};
  const void* hp[1] = {plan->blob.data() + plan->off_poly};
  hipError_t e = pat::run_op(plan->prec, op, 1, &h, dd, hp, ins, outs, wss, nullptr, static_cast<hipStream_t>(stream), tm);
  if (e != hipSuccess) return hip_err(e, "kernel launch");
  return PAT_OK;
}

pat_status run(pat_plan* plan, pat::Op op, const void* in, size_t in_bytes, void* out, size_t out_bytes, void* ws,
               size_t ws_bytes, void* stream) {
  pat_status s = check_call(plan, op, in, in_bytes, out, out_bytes);
  if (s != PAT_OK) return s;
  if (!aligned16(ws)) return set_err(PAT_ERR_WORKSPACE, "workspace NULL or not 16-byte aligned");
  s = check_size("workspace", ws_bytes, plan->ws_bytes, PAT_ERR_WORKSPACE);
  if (s != PAT_OK) return s;
  arm_faults();
  return enqueue(plan, plan->inst, op, in, out, ws, stream, timer_of(plan));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Releases fork streams (HIP errors ignored: this also runs at process exit).
void destroy_fork(pat::ForkStreams* f) {
  if (!f) return;
  for (auto& st : f->s)
    if (st) (void)hipStreamDestroy(st);
  for (auto& ev : f->ev)
    if (ev) (void)hipEventDestroy(ev);
  delete f;
}

}  // namespace

extern "C" {

pat_status pat_plan_create(const pat_geometry* geom, pat_plan** out) {
  if (!geom || !out) return set_err(PAT_ERR_INVALID_ARG, "geometry or output pointer is NULL");
  *out = nullptr;
  pat_plan* p = new (std::nothrow) pat_plan();
  if (!p) return set_err(PAT_ERR_INTERNAL, "out of host memory");
  std::string err;
  pat_status s;
  try {
    s = pat::build_plan(*geom, p, &err);
  } catch (...) {
    s = PAT_ERR_INTERNAL;
    err = "exception while building the plan";
  }
  if (s != PAT_OK) {
    delete p;
    return set_err(s, err);
  }
  *out = p;
  return PAT_OK;
}

pat_status pat_plan_sizes(const pat_plan* plan, size_t* table_bytes, size_t* workspace_bytes) {
  if (!plan) return set_err(PAT_ERR_INVALID_ARG, "plan is NULL");
  if (table_bytes) *table_bytes = plan->table_bytes;
  if (workspace_bytes) *workspace_bytes = plan->ws_bytes;
  return PAT_OK;
}

pat_status pat_plan_upload(pat_plan* plan, void* table_dev, size_t table_bytes, void* stream) {
  if (!plan) return set_err(PAT_ERR_INVALID_ARG, "plan is NULL");
  if (!aligned16(table_dev)) return set_err(PAT_ERR_INVALID_ARG, "table buffer NULL or not 16-byte aligned");
  pat_status s = check_size("table buffer", table_bytes, plan->table_bytes, PAT_ERR_WORKSPACE);
  if (s != PAT_OK) return s;
  const Faults f = arm_faults();
  if (f.upload) return hip_err(hipErrorOutOfMemory, "hipMemcpyAsync(table) [PAT_FAULT=upload]");
  pat::bind_table(plan, table_dev);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(table_dev, plan->blob.data(), plan->table_bytes, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_err(e, "hipMemcpyAsync(table)");
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_err(e, "hipStreamSynchronize");
  plan->uploaded = true;
  return PAT_OK;
}

pat_status pat_reconstruct(pat_plan* plan, const void* p, size_t p_bytes, void* f, size_t f_bytes, void* ws,
                           size_t ws_bytes, void* stream) {
  return run(plan, pat::OP_R, p, p_bytes, f, f_bytes, ws, ws_bytes, stream);
}

pat_status pat_reconstruct_adjoint(pat_plan* plan, const void* f, size_t f_bytes, void* p, size_t p_bytes, void* ws,
                           size_t ws_bytes, void* stream) {
  return run(plan, pat::OP_RT, f, f_bytes, p, p_bytes, ws, ws_bytes, stream);
}

pat_status pat_forward(pat_plan* plan, const void* f, size_t f_bytes, void* p, size_t p_bytes, void* ws,
                           size_t ws_bytes, void* stream) {
  return run(plan, pat::OP_A, f, f_bytes, p, p_bytes, ws, ws_bytes, stream);
}

pat_status pat_forward_adjoint(pat_plan* plan, const void* p, size_t p_bytes, void* f, size_t f_bytes, void* ws,
                           size_t ws_bytes, void* stream) {
  return run(plan, pat::OP_AT, p, p_bytes, f, f_bytes, ws, ws_bytes, stream);
}

pat_status pat_reconstruct_noalloc(pat_plan* plan, const void* p, size_t p_bytes, void* f, size_t f_bytes,
                                   void* stream) {
  pat_status s = check_call(plan, pat::OP_R, p, p_bytes, f, f_bytes);
  if (s != PAT_OK) return s;
  // the fused line path never stores the oversampled grid: its workspace is
  // G and F only, packed back to back
  pat::Inst h = plan->inst;
  const size_t cs = pat::complex_bytes(plan->prec);
  size_t need = plan->ws_bytes;
  if (h.fused) {
    h.off_u = h.off_f = (int64_t)align256((size_t)h.lines * h.nt * cs);
    need = (size_t)h.off_f + align256((size_t)h.lines * h.nz * cs);
  }
  if (need > pat::kScratchBytes)
    return set_err(PAT_ERR_UNSUPPORTED, "this plan needs " + std::to_string(need) +
                                            " bytes of workspace; the static scratch of pat_reconstruct_noalloc holds " +
                                            std::to_string(pat::kScratchBytes));
  const Faults fl = arm_faults();
  if (fl.scratch) return hip_err(hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch) [PAT_FAULT=scratch]");
  void* ws = nullptr;
  hipError_t e = pat::scratch_buffer(&ws);
  if (e != hipSuccess) return hip_err(e, "hipGetSymbolAddress(scratch)");
  // (no stage timing here: recording it creates events)
  return enqueue(plan, h, pat::OP_R, p, f, ws, stream, nullptr);
}

pat_status pat_batched_workspace_size(int32_t n, pat_plan* const* plans, size_t* workspace_bytes) {
  if (!plans || !workspace_bytes) return set_err(PAT_ERR_INVALID_ARG, "NULL argument");
  if (n < 1 || n > pat::kMaxBatch) return set_err(PAT_ERR_INVALID_ARG, "batch size must be in [1, 32]");
  size_t total = align256(pat::kNumCounters * sizeof(uint32_t));
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) return set_err(PAT_ERR_INVALID_ARG, "NULL plan in batch");
    total += align256(plans[i]->ws_bytes);
  }
  *workspace_bytes = total;
  return PAT_OK;
}

// The fork streams of the batched calls whose first plan this is, created on
// the first such call (default priority, non-blocking); nullptr if HIP
// refuses them, and the call then runs on the caller's stream alone.
static const pat::ForkStreams* fork_of(pat_plan* plan) {
  if (plan->fork) return static_cast<const pat::ForkStreams*>(plan->fork);
  auto* f = new pat::ForkStreams;
  bool ok = true;
  for (auto& s : f->s) ok = ok && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
  for (auto& e : f->ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    destroy_fork(f);
    (void)hipGetLastError();
    return nullptr;
  }
  plan->fork = f;
  return f;
}

pat_status pat_reconstruct_batched(int32_t n, pat_plan* const* plans, const void* const* p, const size_t* p_bytes,
                                   void* const* f, const size_t* f_bytes, void* ws, size_t ws_bytes, void* stream) {
  if (!plans || !p || !f || !p_bytes || !f_bytes) return set_err(PAT_ERR_INVALID_ARG, "NULL argument");
  if (n < 1 || n > pat::kMaxBatch) return set_err(PAT_ERR_INVALID_ARG, "batch size must be in [1, 32]");
  if (!aligned16(ws)) return set_err(PAT_ERR_WORKSPACE, "workspace NULL or not 16-byte aligned");
  size_t need = 0;
  pat_status s0 = pat_batched_workspace_size(n, plans, &need);
  if (s0 != PAT_OK) return s0;
  s0 = check_size("workspace", ws_bytes, need, PAT_ERR_WORKSPACE);
  if (s0 != PAT_OK) return s0;
  pat::Inst h[pat::kMaxBatch];
  const pat::Inst* d[pat::kMaxBatch];
  const void* hp[pat::kMaxBatch];
  void* wsi[pat::kMaxBatch];
  unsigned char* w = static_cast<unsigned char*>(ws);
  uint32_t* counters = reinterpret_cast<uint32_t*>(w);
  size_t off = align256(pat::kNumCounters * sizeof(uint32_t));
  for (int i = 0; i < n; ++i) {
    pat_status s = check_plan(plans[i]);
    if (s != PAT_OK) return s;
    if (plans[i]->prec != plans[0]->prec) return set_err(PAT_ERR_INVALID_ARG, "plans in a batch must share a precision");
    if (!aligned16(p[i]) || !aligned16(f[i]))
      return set_err(PAT_ERR_INVALID_ARG, "input/output NULL or not 16-byte aligned");
    s = check_size("input array", p_bytes[i], column_array_bytes(plans[i], false), PAT_ERR_INVALID_ARG);
    if (s != PAT_OK) return s;
    s = check_size("output array", f_bytes[i], column_array_bytes(plans[i], true), PAT_ERR_INVALID_ARG);
    if (s != PAT_OK) return s;
    h[i] = plans[i]->inst;
    hp[i] = plans[i]->blob.data() + plans[i]->off_poly;
    d[i] = reinterpret_cast<const pat::Inst*>(static_cast<unsigned char*>(plans[i]->table_dev) + plans[i]->off_desc);
    wsi[i] = w + off;
    off += align256(plans[i]->ws_bytes);
  }
  arm_faults();
  pat::StageTimer* tm = timer_of(plans[0]);
  hipError_t e = pat::run_op(plans[0]->prec, pat::OP_R, n, h, d, hp, p, f, wsi, counters,
                             static_cast<hipStream_t>(stream), tm, n > 1 && !tm ? fork_of(plans[0]) : nullptr);
  if (e != hipSuccess) return hip_err(e, "kernel launch");
  return PAT_OK;
}

// Bytes of the line-stage arrays: the oversampled grid (lines x c nt, grid
// storage) and the node values (lines x nz complex).
size_t grid_array_bytes(const pat_plan* p) { return (size_t)p->inst.lines * p->inst.m * pat::grid_bytes(p->prec); }
size_t values_array_bytes(const pat_plan* p) {
  return (size_t)p->inst.lines * p->inst.nz * pat::complex_bytes(p->prec);
}

pat_status pat_nufft2_lines(pat_plan* plan, const void* grid, size_t grid_bytes, void* out, size_t out_bytes,
                            void* stream) {
  pat_status s = check_plan(plan);
  if (s != PAT_OK) return s;
  if (!aligned16(grid) || !aligned16(out)) return set_err(PAT_ERR_INVALID_ARG, "grid/out NULL or not 16-byte aligned");
  s = check_size("grid array", grid_bytes, grid_array_bytes(plan), PAT_ERR_INVALID_ARG);
  if (s != PAT_OK) return s;
  s = check_size("output array", out_bytes, values_array_bytes(plan), PAT_ERR_INVALID_ARG);
  if (s != PAT_OK) return s;
  const pat::Inst* d = reinterpret_cast<const pat::Inst*>(static_cast<unsigned char*>(plan->table_dev) + plan->off_desc);
  arm_faults();
  hipError_t e = pat::run_interp(plan->prec, plan->inst, d, plan->blob.data() + plan->off_poly, grid, out,
                                 static_cast<hipStream_t>(stream), timer_of(plan));
  if (e != hipSuccess) return hip_err(e, "kernel launch");
  return PAT_OK;
}

pat_status pat_nufft1_lines(pat_plan* plan, const void* values, size_t values_bytes, void* grid, size_t grid_bytes,
                            void* stream) {
  pat_status s = check_plan(plan);
  if (s != PAT_OK) return s;
  if (!aligned16(values) || !aligned16(grid)) return set_err(PAT_ERR_INVALID_ARG, "values/grid NULL or not 16-byte aligned");
  s = check_size("values array", values_bytes, values_array_bytes(plan), PAT_ERR_INVALID_ARG);
  if (s != PAT_OK) return s;
  s = check_size("grid array", grid_bytes, grid_array_bytes(plan), PAT_ERR_INVALID_ARG);
  if (s != PAT_OK) return s;
  if (plan->inst.kind != PAT_INTERP_KB)
    return set_err(PAT_ERR_UNSUPPORTED, "spreading needs interp = PAT_INTERP_KB");
  if (!plan->spread_ok) return set_err(PAT_ERR_UNSUPPORTED, "nz too large for the spreading lists of a depth line in LDS");
  const pat::Inst* d = reinterpret_cast<const pat::Inst*>(static_cast<unsigned char*>(plan->table_dev) + plan->off_desc);
  arm_faults();
  hipError_t e = pat::run_spread(plan->prec, plan->inst, d, plan->blob.data() + plan->off_poly, values, grid,
                                 static_cast<hipStream_t>(stream), timer_of(plan));
  if (e != hipSuccess) return hip_err(e, "kernel launch");
  return PAT_OK;
}

pat_status pat_plan_set_fused(pat_plan* plan, int32_t fused) {
  if (!plan) return set_err(PAT_ERR_INVALID_ARG, "plan is NULL");
  if (fused && !plan->fusable) return set_err(PAT_ERR_UNSUPPORTED, "this plan cannot run the fused line kernels");
  // the launchers choose kernels from the host copy of the descriptor
  plan->inst.fused = fused ? 1 : 0;
  return PAT_OK;
}

pat_status pat_plan_set_timing(pat_plan* plan, int32_t on) {
  if (!plan) return set_err(PAT_ERR_INVALID_ARG, "plan is NULL");
  plan->timing = on != 0;
  return PAT_OK;
}

pat_status pat_plan_stage_times(pat_plan* plan, int32_t cap, const char** names, float* ms, int32_t* count) {
  if (!plan || !count) return set_err(PAT_ERR_INVALID_ARG, "NULL argument");
  *count = 0;
  EventTimer* t = static_cast<EventTimer*>(plan->timer);
  if (!t) return PAT_OK;
  const int n = t->count();
  for (int i = 0; i < n && i < cap; ++i) {
    if (names) names[i] = t->name(i);
    if (ms) ms[i] = t->ms(i);
  }
  *count = n;
  t->reset();
  return PAT_OK;
}

void pat_plan_destroy(pat_plan* plan) {
  if (!plan) return;
  destroy_fork(static_cast<pat::ForkStreams*>(plan->fork));
  delete static_cast<EventTimer*>(plan->timer);
  delete plan;
}

const char* pat_status_string(pat_status s) {
  switch (s) {
    case PAT_OK: return "PAT_OK";
    case PAT_ERR_INVALID_ARG: return "PAT_ERR_INVALID_ARG";
    case PAT_ERR_UNSUPPORTED: return "PAT_ERR_UNSUPPORTED";
    case PAT_ERR_WORKSPACE: return "PAT_ERR_WORKSPACE";
    case PAT_ERR_HIP: return "PAT_ERR_HIP";
    case PAT_ERR_INTERNAL: return "PAT_ERR_INTERNAL";
  }
  return "PAT_ERR_UNKNOWN";
}

const char* pat_last_error(void) { return g_err.c_str(); }

}  // extern "C"
