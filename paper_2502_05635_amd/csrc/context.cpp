// Context lifetime, error reporting, workspace and profiling events.
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>

#include "internal.h"

static std::string g_create_err;

namespace tdg {

int fail(tdg_ctx ctx, int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx)
    ctx->err = buf;
  else
    g_create_err = buf;
  return code;
}

int hip_check(tdg_ctx ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return TDG_OK;
  return fail(ctx, TDG_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

int launch_check(tdg_ctx ctx, const char* what) { return hip_check(ctx, hipGetLastError(), what); }

int ws_reserve(tdg_ctx ctx, WsSlot slot, size_t bytes, void** out) {
  Buf& b = ctx->ws[slot];
  if (bytes == 0) bytes = 256;
  if (b.bytes < bytes) {
    if (b.p) {
      // the old buffer may still be read by queued work
      hipError_t e = hipStreamSynchronize(ctx->stream);
      if (e != hipSuccess) return hip_check(ctx, e, "workspace resize sync");
      hipFree(b.p);
      b.p = nullptr;
      b.bytes = 0;
    }
    size_t want = (bytes + 255) & ~size_t(255);
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
      b.p = nullptr;
      return fail(ctx, TDG_E_NOMEM, "workspace slot %d: cannot allocate %zu bytes (%s)", int(slot), want,
                  hipGetErrorString(e));
    }
    b.bytes = want;
  }
  *out = b.p;
  return TDG_OK;
}

void prof_begin(tdg_ctx ctx, int kclass) {
  if (!ctx->prof) return;
  auto& v = ctx->events[kclass];
  size_t i = ctx->used[kclass];
  if (i == v.size()) {
    EventPair p;
    if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) return;
    v.push_back(p);
  }
  hipEventRecord(v[i].a, ctx->stream);
}

void prof_end(tdg_ctx ctx, int kclass) {
  if (!ctx->prof) return;
  auto& v = ctx->events[kclass];
  size_t i = ctx->used[kclass];
  if (i >= v.size()) return;
  hipEventRecord(v[i].b, ctx->stream);
  ctx->used[kclass] = i + 1;
}

void prof_pair(tdg_ctx ctx, int kclass, hipEvent_t* a, hipEvent_t* b) {
  *a = *b = nullptr;
  if (!ctx->prof) return;
  auto& v = ctx->events[kclass];
  size_t i = ctx->used[kclass];
  if (i == v.size()) {
    EventPair p;
    if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) return;
    v.push_back(p);
  }
  *a = v[i].a;
  *b = v[i].b;
  ctx->used[kclass] = i + 1;
}

int pairs_per_k(const tdg_model* m, int block) {
  if (block == TDG_BLOCK_ALL) return m->nb * m->nb;
  if (block == TDG_BLOCK_EH) return (m->nb - m->nv) * m->nv;
  return -1;
}

int validate_model(tdg_ctx ctx, const tdg_model* m) {
  if (!m) return fail(ctx, TDG_E_INVAL, "model is NULL");
  if (m->nk1 <= 0 || m->nk2 <= 0) return fail(ctx, TDG_E_INVAL, "grid %d x %d must be positive", m->nk1, m->nk2);
  if (m->nb < 2 || m->nb > TDG_NB_MAX)
    return fail(ctx, TDG_E_INVAL, "nb = %d outside [2, %d]", m->nb, TDG_NB_MAX);
  if (m->nv < 1 || m->nv >= m->nb) return fail(ctx, TDG_E_INVAL, "nv = %d outside [1, nb-1]", m->nv);
  if (!(m->a_bohr > 0.0)) return fail(ctx, TDG_E_INVAL, "lattice constant must be positive");
  if (!m->eps || !m->evec || !m->dip || !m->vel) return fail(ctx, TDG_E_INVAL, "model array pointer is NULL");
  if (((uintptr_t)m->evec | (uintptr_t)m->dip | (uintptr_t)m->vel | (uintptr_t)m->links) & 15)
    return fail(ctx, TDG_E_INVAL, "complex model arrays must be 16-byte aligned");
  return TDG_OK;
}

}  // namespace tdg

using namespace tdg;

extern "C" {

int tdg_version(void) { return 100; }

int tdg_create(tdg_ctx* out, int device, void* hip_stream) {
  if (!out) return fail(nullptr, TDG_E_INVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return fail(nullptr, TDG_E_HIP, "hipGetDeviceCount: %s", hipGetErrorString(e));
  if (device < 0 || device >= count) return fail(nullptr, TDG_E_INVAL, "device %d of %d", device, count);
  e = hipSetDevice(device);
  if (e != hipSuccess) return fail(nullptr, TDG_E_HIP, "hipSetDevice: %s", hipGetErrorString(e));
  TDG_TRY(scratch_init(device));
  tdg_ctx c = new (std::nothrow) tdg_ctx_s();
  if (!c) return fail(nullptr, TDG_E_NOMEM, "context allocation");
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  *out = c;
  return TDG_OK;
}

int tdg_destroy(tdg_ctx ctx) {
  if (!ctx) return TDG_OK;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  for (auto& b : ctx->ws)
    if (b.p) hipFree(b.p);
  for (auto& v : ctx->events)
    for (auto& p : v) {
      hipEventDestroy(p.a);
      hipEventDestroy(p.b);
    }
  release_blas(ctx);
  if (ctx->order_ev) hipEventDestroy(ctx->order_ev);
  delete ctx;
  return TDG_OK;
}

int tdg_set_stream(tdg_ctx ctx, void* hip_stream) {
  if (!ctx) return TDG_E_INVAL;
  const hipStream_t next = (hipStream_t)hip_stream;
  if (next == ctx->stream) return TDG_OK;
  // work queued on the old stream still reads and writes the context's
  // workspace: the new stream waits for it before anything queued after
  TDG_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
  if (!ctx->order_ev)
    TDG_TRY(hip_check(ctx, hipEventCreateWithFlags(&ctx->order_ev, hipEventDisableTiming), "stream order event"));
  TDG_TRY(hip_check(ctx, hipEventRecord(ctx->order_ev, ctx->stream), "stream order record"));
  TDG_TRY(hip_check(ctx, hipStreamWaitEvent(next, ctx->order_ev, 0), "stream order wait"));
  ctx->stream = next;
  return TDG_OK;
}

const char* tdg_last_error(tdg_ctx ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

int tdg_set_option(tdg_ctx ctx, int32_t option, int64_t value) {
  if (!ctx) return TDG_E_INVAL;
  if (option == TDG_OPT_AUTOTUNE) {
    ctx->autotune = value != 0;
    return TDG_OK;
  }
  if (option == TDG_OPT_BATCHED_MIN) {
    if (value < 1) return fail(ctx, TDG_E_INVAL, "batched minimum must be >= 1");
    ctx->batched_min = (int)std::min<int64_t>(value, 1 << 30);
    return TDG_OK;
  }
  if (option == TDG_OPT_GEMM_TILE) {
    if (value != 64 && value != 128) return fail(ctx, TDG_E_INVAL, "GEMM tile must be 64 or 128");
    ctx->gemm_variant = value == 64 ? 0 : 2;
    return TDG_OK;
  }
  if (option == TDG_OPT_GRAPHS) {
    ctx->graphs = value != 0;
    return TDG_OK;
  }
  if (option == TDG_OPT_ADJOINT_STASH) {
    if (value < 0 || value > 2) return fail(ctx, TDG_E_INVAL, "adjoint stash %lld is not 0, 1 or 2", (long long)value);
    ctx->adj_stash = (int)value;
    return TDG_OK;
  }
  if (option == TDG_OPT_GEMM_SLICES) {
    if (value < 0 || value > 4096) return fail(ctx, TDG_E_INVAL, "GEMM slices %lld outside [0, 4096]", (long long)value);
    ctx->gemm_slices = (int)value;
    return TDG_OK;
  }
  if (option == TDG_OPT_GEMM_VARIANT) {
    if (value < -1 || value > 4) return fail(ctx, TDG_E_INVAL, "GEMM variant %lld outside [-1, 4]", (long long)value);
    ctx->gemm_variant = (int)value;
    return TDG_OK;
  }
  if (option == TDG_OPT_STAGE_VARIANT) {
    if (value < -1 || value > 64) return fail(ctx, TDG_E_INVAL, "variant index %lld", (long long)value);
    ctx->forced_variant = (int)value;
    return TDG_OK;
  }
  return fail(ctx, TDG_E_INVAL, "unknown option %d", option);
}

const char* tdg_last_variant(tdg_ctx ctx) { return ctx ? ctx->last_variant.c_str() : ""; }

int tdg_profile_enable(tdg_ctx ctx, int32_t on) {
  if (!ctx) return TDG_E_INVAL;
  ctx->prof = on != 0;
  for (auto& u : ctx->used) u = 0;
  return TDG_OK;
}

int tdg_profile_read(tdg_ctx ctx, int32_t kclass, double* total_ms, int64_t* launches) {
  if (!ctx) return TDG_E_INVAL;
  if (kclass < 0 || kclass >= KCLASS_COUNT || !total_ms || !launches)
    return fail(ctx, TDG_E_INVAL, "profile_read: bad class or NULL output");
  TDG_TRY(hip_check(ctx, hipStreamSynchronize(ctx->stream), "profile sync"));
  double tot = 0.0;
  auto& v = ctx->events[kclass];
  for (size_t i = 0; i < ctx->used[kclass]; ++i) {
    float ms = 0.f;
    TDG_TRY(hip_check(ctx, hipEventElapsedTime(&ms, v[i].a, v[i].b), "hipEventElapsedTime"));
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)ctx->used[kclass];
  return TDG_OK;
}

}  // extern "C"
