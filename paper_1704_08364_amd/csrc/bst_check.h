// bst_check.h -- index checks of the checked build (BST_CHECKED defined):
// every use of BST_IDX(i, n, bit) verifies 0 <= i < n; a failing index sets
// `bit` in the module's flag word (a vector atomic on global memory) and is
// replaced by 0, so the access stays in bounds and the kernel runs to its end.
// The host reads and clears the flags through bst_debug_check. Release builds
// compile BST_IDX to its index and contain no flag.
#pragma once

#include "bst_internal.h"

#ifdef BST_CHECKED

namespace bst {
// one flag word per compiled module (internal linkage)
static __device__ unsigned g_check_flags;

template <typename I, typename N>
__device__ __forceinline__ I checked_index(I i, N n, unsigned bit) {
    if ((unsigned long long)i >= (unsigned long long)n) {
        atomicOr(&g_check_flags, 1u << bit);
        return (I)0;
    }
    return i;
}
}  // namespace bst

#define BST_IDX(i, n, bit) ::bst::checked_index((i), (n), (bit))

// host reader of this module's flags (reads and clears)
#define BST_CHECK_MODULE(name)                                                                  \
    namespace bst {                                                                             \
    unsigned check_flags_##name() {                                                             \
        unsigned v = 0, zero = 0;                                                               \
        if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_check_flags), sizeof(v)) != hipSuccess) return ~0u; \
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_check_flags), &zero, sizeof(zero)) != hipSuccess) return ~0u; \
        return v;                                                                               \
    }                                                                                           \
    }

#else

#define BST_IDX(i, n, bit) (i)
#define BST_CHECK_MODULE(name)

#endif
