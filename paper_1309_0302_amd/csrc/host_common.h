// Host-side helpers shared by the single-problem and batched ABI files.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/godec.h"

namespace godec_host {

// Message of the calling thread's last failure (godec_last_error).
extern thread_local std::string g_last_error;

inline godec_status fail(godec_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over the workspace (base == nullptr only measures).
struct Carver {
  char* base;
  size_t off = 0;
  void* take(size_t bytes) {
    off = align_up(off, 256);
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

int device_cu_count();

// Padded shapes and tilings of the panel passes over an m x n matrix (k: the
// cardinality bound, which sizes the candidate buffer of the sparse step).
struct PanelPlan {
  int64_t ldd, mpad, nchunks, rpc, cap;
  int64_t kc_a, nct_a, rc_b, nch_b;   // matrix-core tilings
};
PanelPlan plan_sizes(int64_t m, int64_t n, int64_t k, int num_cu);

// Enqueue (on the batch's stream) a copy of every problem's current S list:
// problem i's entries, in selection order, to idx_dev/val_dev + i * kstride,
// and its length to nnz_dev[i].
godec_status batch_snapshot_S(godec_batch* b, int64_t* idx_dev, float* val_dev, int64_t kstride,
                              int64_t* nnz_dev);

// Current rank of every problem of the batch (one copy, synchronises the
// batch's stream).
godec_status batch_ranks(godec_batch* b, int* rank_host);

// Enqueue a copy of every problem's factors U_L (m x r) and V_L (n x r) to
// U_dev + i sU and V_dev + i sV (one launch on the batch's stream).
godec_status batch_factors(godec_batch* b, float* U_dev, int64_t sU, float* V_dev, int64_t sV);

}  // namespace godec_host

#define HIP_TRY(expr)                                                        \
  do {                                                                       \
    hipError_t _e = (expr);                                                  \
    if (_e != hipSuccess)                                                    \
      return godec_host::fail(GODEC_E_DEVICE,                                \
                              std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)
