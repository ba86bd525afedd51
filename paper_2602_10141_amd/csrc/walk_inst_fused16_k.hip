// Instantiation of the fused Gray walk kernel (walk_impl.h): orders <= 16, Kahan sums.
#include "walk_impl.h"

namespace permk {

WalkFn walk_fn_fused16_k() { return &walk_fused<16, true>; }

}  // namespace permk
