// Instantiation of the fused Gray walk kernel (walk_impl.h): orders <= 16, plain sums.
#include "walk_impl.h"

namespace permk {

WalkFn walk_fn_fused16_nok() { return &walk_fused<16, false>; }

}  // namespace permk
