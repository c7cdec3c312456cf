// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <string>
#include <vector>

#include "tdagw.h"

namespace tdg {

// Workspace slots owned by a context (grow-only device allocations).
enum WsSlot {
  WS_RHO_S = 0,  // stage state          c128 [B][nk][nb][nb]
  WS_ACC,        // RK4 accumulator      c128 [B][nk][nb][nb]
  WS_X0,         // drho gather, ping    [B][N] (operator dtype)
  WS_X1,         // drho gather, pong
  WS_Z,          // low-rank projection  [B][r]
  WS_OBS_PART,   // per-k observables    double [chunk][B][nk][5]
  WS_FIELDS,     // field records        tdg_field [B], then the sorted -> caller's instance map int [B]
  WS_WTAB,       // W(q) by index difference, double [nk1][nk2]
  WS_SOLVER_A,   // compression: K_off column-major, c128 [n][n]
  WS_SOLVER_D,   // eigenvalues / off-diagonal, double [2n]
  WS_SOLVER_I,   // info, permutation, kept eigenvalues
  WS_MISC,       // small scratch (row sums, flags)
  WS_RHO_N,      // rho(t_n) in sorted instance order, c128 [B][nk][nb][nb]
  WS_Y,          // batched: contraction result / split-K partials, c64
  WS_ZSUM,       // batched low rank: projection summed over its split-K slices, c64
  WS_TMP1,       // conversion staging (complex64 copies before a BF16X2 split)
  WS_TMP2,
  WS_TMP3,
  WS_RSVD_Y,     // randomized compression: range block, then Q, c128 column-major [l][n]
  WS_RSVD_Z,     // randomized compression: K_off Q, then Q W, c128 column-major [l][n]
  WS_RSVD_F,     // randomized compression: complex64 copies of Q and K Q for a C64 kernel
  WS_RSVD_T,     // randomized compression: Q^H K_off Q, c128 [l][l], and Householder scalars
  WS_ADJ,        // adjoint propagation: checkpoints, segment states, stage data, cotangents
  WS_STEP,       // batched path: step counter read by graph replays
  WS_XB,         // batched BF16X2 path: X split into bf16 planes once per product
  WS_INTRA,      // intraband term: covariant derivative of the stage state, c128 like the state
  WS_RHO_S2,     // intraband term, per-instance path: second stage-state buffer (stages alternate)
  WS_FTAB,       // field at the stage times of a chunk of steps, double [chunk][B][4]
  WS_XE,         // batched BF16X2 path: the gather split by the stage kernel for the next product
  WS_COUNT
};

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
};

constexpr int KCLASS_COUNT = 4;  // TDG_KCLASS_STAGE .. TDG_KCLASS_INTRA

}  // namespace tdg

struct tdg_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  tdg::Buf ws[tdg::WS_COUNT];
  void* blas = nullptr;  // rocblas_handle, created on first compression
  bool prof = false;
  std::vector<tdg::EventPair> events[tdg::KCLASS_COUNT];
  size_t used[tdg::KCLASS_COUNT] = {};
  // stage-kernel variant selection (see tdg_set_option)
  bool autotune = true;
  int forced_variant = -1;
  int batched_min = 4;  // complex64 operators use the matrix-core path from this batch size
  int gemm_variant = -1; // tiling of the matrix-core product: -1 tuned per shape, else 0..2 (cgemm_f32)
  bool graphs = false;   // replay captured steps or chunks (TDG_OPT_GRAPHS)
  int gemm_slices = 0;   // batched products: 0 = tuned split-K, else this many K slices (TDG_OPT_GEMM_SLICES)
  int adj_stash = 2;     // adjoint: keep the whole run's or a segment's stage data when it fits (TDG_OPT_ADJOINT_STASH)
  hipEvent_t order_ev = nullptr;  // tdg_set_stream: orders the new stream after the old one's queued work
  std::vector<std::pair<std::string, int>> tuned;  // shape key -> variant index
  std::string last_variant;
};

namespace tdg {

int fail(tdg_ctx ctx, int code, const char* fmt, ...);
// Ensure workspace slot holds at least `bytes`; returns TDG_OK or an error.
int ws_reserve(tdg_ctx ctx, WsSlot slot, size_t bytes, void** out);
// Check the last launch / HIP status and convert to a library error.
int hip_check(tdg_ctx ctx, hipError_t e, const char* what);
int launch_check(tdg_ctx ctx, const char* what);
// Profiling brackets (no-ops unless profiling is on).
void prof_begin(tdg_ctx ctx, int kclass);
void prof_end(tdg_ctx ctx, int kclass);
// Events for one kernel launched with hipExtLaunchKernelGGL (timestamps of the
// dispatch itself); both NULL unless profiling is on.
void prof_pair(tdg_ctx ctx, int kclass, hipEvent_t* a, hipEvent_t* b);
int validate_model(tdg_ctx ctx, const tdg_model* m);
int pairs_per_k(const tdg_model* m, int block);
// Destroy the context's rocBLAS handle if compression created one.
void release_blas(tdg_ctx ctx);
// The context's rocBLAS handle (created on first use), bound to its stream.
int blas_handle(tdg_ctx ctx, void** handle);
// Complex FP32 matrix-core product Y[s] = A * X over split-K slices s (gemm.hip);
// variant 0 = 64-row tiles, 1 = 64-row tiles with a prefetched next tile, 2 =
// 128-row tiles.
void cgemm_f32(hipStream_t stream, const void* A, int64_t lda, int M, int Kc, const void* X, int64_t ldx, void* Y,
               int64_t ldy, int64_t y_slice_stride, int ncols, int kslice, int variant);
// BF16 split-precision product: A in TDG_BF16X2 storage (hi plane, then lo
// plane, [M][lda], lda % 4 == 0), X complex64 [Kc][ldx] (gemm.hip).
// variant 0: 64-row tiles splitting X while staged; 1 to 4: X split once
// into `work` (cgemm_bf16x2_work_bytes bytes), then 128-row tiles (1),
// 256-row tiles staged by direct-to-LDS loads (2), 128-row tiles of 64 real
// K per stage (3), or 128-row tiles staged by direct-to-LDS loads (4).
void cgemm_bf16x2(hipStream_t stream, const void* A, int64_t lda, int M, int Kc, const void* X, int64_t ldx,
                  void* Y, int64_t ldy, int64_t y_slice_stride, int ncols, int kslice, int variant, void* work,
                  bool x_expanded = false);
// The split X of BF16X2 tilings 1 to 4 (complex64 [Kc][ldx], first ncols
// instances; the rest of the last tile zero) written into `work`.
void expand_bf16x2(hipStream_t stream, const void* X, int64_t ldx, int Kc, int ncols, void* work);
// The split X of BF16X2 tilings 1 to 4 written into `work` straight from
// `slices` split-K partial products (complex64 [Kc][ldx] each, `stride`
// apart; ldx and stride even), summed in slice order: then call cgemm_bf16x2
// with x_expanded (X unused).
void sum_expand_bf16x2(hipStream_t stream, const void* in, int slices, int64_t stride, int Kc, int64_t ldx, int ncols,
                       void* work);
size_t cgemm_bf16x2_work_bytes(int Kc, int ncols);
// dst (TDG_BF16X2 [rows][ld_dst]) <- complex src [rows][ld_src]; columns >= cols zero.
void split_bf16x2(hipStream_t stream, const void* src, int src_is_double, int64_t ld_src, int64_t rows, int64_t cols,
                  void* dst, int64_t ld_dst);
// out = e.(y)_{;k} per instance (intraband.hip): the covariant k-derivative of
// the per-k matrices y with model->links, y and out addressed as
// b*sb + k*sk + e*se (element e = n*nb + m), e taken from fields[b] (device).
// Launch only (no error check: also used under graph capture); the caller
// keeps nk * nb^2 * batch at most 2^38 (the grid limit).  ea / eb: dispatch
// timestamp events (prof_pair) or NULL.
void covariant_derivative(hipStream_t stream, const tdg_model* model, const void* y, int64_t sb, int64_t sk,
                          int64_t se, const tdg_field* fields, int batch, void* out, hipEvent_t ea = nullptr,
                          hipEvent_t eb = nullptr);
// out = sum of `slices` complex64 arrays of `count` elements, `stride` apart
// (count, stride even; in and out 16-byte aligned).
void sum_slices_c64(hipStream_t stream, const void* in, int slices, int64_t stride, int64_t count, void* out);
// Copy `bytes` (a multiple of 4) of host memory to device memory `dev`
// (4-byte aligned) inside the arguments of kernels queued on the context
// stream: the call does not wait, and the host array need not outlive it.
int args_upload(tdg_ctx ctx, void* dev, const void* host, size_t bytes);
// Look up, once per device (the device current), the device address of the
// scratch array of tdg_propagate_noalloc (propagate.hip).
int scratch_init(int device);

}  // namespace tdg

#define TDG_TRY(expr)              \
  do {                             \
    int _rc = (expr);              \
    if (_rc != TDG_OK) return _rc; \
  } while (0)
