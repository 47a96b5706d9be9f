// Launch tuning shared by the C ABI and the autotuner (tune.hip).
#pragma once
#include "../../include/sigkernel.h"

namespace sk {

// Key of a call as the public table sees it.
sk_tune_key tune_key_of(int32_t op, const sk_paths* X, const sk_paths* Y, int32_t lam,
                        uint32_t flags);

// The tuning a call uses: the candidate being timed by sigkernel_autotune on
// this thread, else the table's entry for the call's key, else all zeros
// (the built-in rules).
sk_tune tuning_for(int32_t op, const sk_paths* X, const sk_paths* Y, int32_t lam,
                   uint32_t flags);

}  // namespace sk
