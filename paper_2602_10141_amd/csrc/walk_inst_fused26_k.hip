// Instantiation of the fused Gray walk kernel (walk_impl.h): orders <= 26, Kahan sums.
#include "walk_impl.h"

namespace permk {

WalkFn walk_fn_fused26_k() { return &walk_fused<26, true>; }

}  // namespace permk
