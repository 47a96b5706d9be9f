// Launch-tuning table and autotuner.  A tuning only changes how pairs are
// spread over waves, workgroups and CUs (include/sigkernel.h lists the
// fields); each pair's arithmetic, and so every output bit, is the same
// under all of them.
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"
#include "tune.h"

namespace {

struct Entry {
  sk_tune_key key;
  sk_tune tune;
};

std::mutex g_mu;
std::vector<Entry> g_table;
thread_local const sk_tune* t_candidate = nullptr;

bool same_key(const sk_tune_key& a, const sk_tune_key& b) {
  return a.op == b.op && a.dyadic_order == b.dyadic_order && a.symmetric == b.symmetric &&
         a.ragged == b.ragged && a.nx == b.nx && a.ny == b.ny && a.x_len == b.x_len &&
         a.y_len == b.y_len && a.dim == b.dim;
}

bool valid_tune(const sk_tune& t) {
  return t.run >= 0 && t.run <= 1024 &&
         (t.waves_per_block == 0 || t.waves_per_block == 1 || t.waves_per_block == 2 ||
          t.waves_per_block == 4) &&
         t.pair_blocks_per_cu >= 0 && t.pair_blocks_per_cu <= 64 && t.pair_bands >= 0 &&
         t.pair_bands <= 1;
}

// The forward call an autotuning candidate is timed on.
sk_status run_call(int32_t op, const sk_paths* X, const sk_paths* Y, int32_t lam, uint32_t flags,
                   float* out, void* ws, size_t ws_bytes, void* stream) {
  return op == SK_OP_PAIR ? sigkernel_pair(X, Y, lam, flags, out, ws, ws_bytes, stream)
                          : sigkernel_gram(X, Y, lam, flags, out, ws, ws_bytes, stream);
}

// Candidate tunings of a forward call: the knobs its launch path reads.
std::vector<sk_tune> candidates(int32_t op, const sk_paths* X, const sk_paths* Y, int32_t lam) {
  std::vector<sk_tune> c;
  // orders beyond the compiled ones run at order 3 on a refined batch with
  // the same fine rows
  const int64_t fine_rows = (int64_t)(X->len > 1 ? X->len - 1 : 1) << lam;
  const bool pair_path = op == SK_OP_PAIR ||
                         sk::choose_rows_per_lane(fine_rows, lam > 3 ? 3 : lam, X->dim) == 0;
  if (pair_path) {
    for (int b : {0, 1, 2, 3, 4, 6, 8}) c.push_back(sk_tune{0, 0, b, 0});
    for (int b : {0, 2, 4}) c.push_back(sk_tune{0, 0, b, 1});  // sequential bands
    return c;
  }
  std::vector<int> runs;
  if (Y->offsets) {
    runs.push_back(1);  // ragged y batches stream one pair per wave
  } else {
    for (int r = 1; r <= 64; r *= 2)
      if (r <= Y->n_paths) runs.push_back(r);
  }
  for (int r : runs)
    for (int w : {1, 2, 4}) c.push_back(sk_tune{r, w, 0, 0});
  return c;
}

}  // namespace

namespace sk {

sk_tune_key tune_key_of(int32_t op, const sk_paths* X, const sk_paths* Y, int32_t lam,
                        uint32_t flags) {
  sk_tune_key k{};
  k.op = op;
  k.dyadic_order = lam;
  k.symmetric = (flags & SK_SYMMETRIC) ? 1 : 0;
  k.ragged = (X->offsets || Y->offsets) ? 1 : 0;
  k.nx = X->n_paths;
  k.ny = Y->n_paths;
  k.x_len = X->len;
  k.y_len = Y->len;
  k.dim = X->dim;
  return k;
}

sk_tune tuning_for(int32_t op, const sk_paths* X, const sk_paths* Y, int32_t lam,
                   uint32_t flags) {
  if (t_candidate) return *t_candidate;
  const sk_tune_key k = tune_key_of(op, X, Y, lam, flags);
  std::lock_guard<std::mutex> lock(g_mu);
  for (const Entry& e : g_table)
    if (same_key(e.key, k)) return e.tune;
  return sk_tune{};
}

}  // namespace sk

extern "C" {

sk_status sigkernel_tune_key(int32_t op, const sk_paths* X, const sk_paths* Y,
                             int32_t dyadic_order, uint32_t flags, sk_tune_key* key) {
  if (!X || !Y || !key) return SK_ERR_NULL;
  if (op != SK_OP_PAIR && op != SK_OP_GRAM && op != SK_OP_GRAM_BACKWARD) return SK_ERR_FLAGS;
  *key = sk::tune_key_of(op, X, Y, dyadic_order, flags);
  return SK_OK;
}

sk_status sigkernel_tune_set(const sk_tune_key* key, const sk_tune* tune) {
  if (!key) return SK_ERR_NULL;
  if (tune && !valid_tune(*tune)) return SK_ERR_FLAGS;
  std::lock_guard<std::mutex> lock(g_mu);
  for (size_t i = 0; i < g_table.size(); ++i) {
    if (!same_key(g_table[i].key, *key)) continue;
    if (tune) {
      g_table[i].tune = *tune;
    } else {
      g_table.erase(g_table.begin() + (std::ptrdiff_t)i);
    }
    return SK_OK;
  }
  if (tune) {
    try {
      g_table.push_back(Entry{*key, *tune});
    } catch (const std::bad_alloc&) {
      return SK_ERR_HIP;
    }
  }
  return SK_OK;
}

int32_t sigkernel_tune_get(const sk_tune_key* key, sk_tune* tune) {
  if (!key || !tune) return SK_ERR_NULL;
  std::lock_guard<std::mutex> lock(g_mu);
  for (const Entry& e : g_table) {
    if (same_key(e.key, *key)) {
      *tune = e.tune;
      return 1;
    }
  }
  return 0;
}

int64_t sigkernel_tune_list(sk_tune_key* keys, sk_tune* tunes, int64_t capacity) {
  std::lock_guard<std::mutex> lock(g_mu);
  const int64_t n = (int64_t)g_table.size();
  for (int64_t i = 0; i < n && i < capacity; ++i) {
    if (keys) keys[i] = g_table[(size_t)i].key;
    if (tunes) tunes[i] = g_table[(size_t)i].tune;
  }
  return n;
}

void sigkernel_tune_clear(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_table.clear();
}

sk_status sigkernel_autotune(int32_t op, const sk_paths* X, const sk_paths* Y,
                             int32_t dyadic_order, uint32_t flags, float* out, void* ws,
                             size_t ws_bytes, int32_t reps, void* stream, sk_tune* best,
                             float* best_ms) {
  if (!X || !Y || !best) return SK_ERR_NULL;
  if (op != SK_OP_PAIR && op != SK_OP_GRAM) return SK_ERR_FLAGS;
  if (reps < 1) return SK_ERR_FLAGS;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) return SK_ERR_HIP;
  if (cap != hipStreamCaptureStatusNone) return SK_ERR_STATE;
  // the call itself must be valid under the built-in rules
  sk_status s = run_call(op, X, Y, dyadic_order, flags, out, ws, ws_bytes, stream);
  if (s != SK_OK) return s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return SK_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return SK_ERR_HIP;
  }
  float best_t = -1.0f;
  sk_tune chosen{};
  s = SK_OK;
  for (const sk_tune& c : candidates(op, X, Y, dyadic_order)) {
    t_candidate = &c;
    sk_status cs = run_call(op, X, Y, dyadic_order, flags, out, ws, ws_bytes, stream);
    float t_min = -1.0f;
    for (int32_t r = 0; cs == SK_OK && r < reps; ++r) {
      if (hipEventRecord(e0, st) != hipSuccess) {
        cs = SK_ERR_HIP;
        break;
      }
      cs = run_call(op, X, Y, dyadic_order, flags, out, ws, ws_bytes, stream);
      if (cs != SK_OK) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        cs = SK_ERR_HIP;
        break;
      }
      if (t_min < 0.0f || ms < t_min) t_min = ms;
    }
    t_candidate = nullptr;
    if (cs == SK_ERR_WORKSPACE || cs == SK_ERR_UNSUPPORTED) continue;  // not for this call
    if (cs != SK_OK) {
      s = cs;
      break;
    }
    if (best_t < 0.0f || t_min < best_t) {
      best_t = t_min;
      chosen = c;
    }
  }
  t_candidate = nullptr;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (s != SK_OK) return s;
  if (best_t < 0.0f) return SK_ERR_UNSUPPORTED;
  const sk_tune_key key = sk::tune_key_of(op, X, Y, dyadic_order, flags);
  if ((s = sigkernel_tune_set(&key, &chosen)) != SK_OK) return s;
  *best = chosen;
  if (best_ms) *best_ms = best_t;
  return SK_OK;
}

}  // extern "C"
