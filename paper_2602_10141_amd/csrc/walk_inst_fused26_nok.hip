// Instantiation of the fused Gray walk kernel (walk_impl.h): orders <= 26, plain sums.
#include "walk_impl.h"

namespace permk {

WalkFn walk_fn_fused26_nok() { return &walk_fused<26, false>; }

}  // namespace permk
