// Instantiations of the Gray walk kernel (walk_impl.h): c128 lo.
#include "walk_impl.h"

namespace permk {

WalkFn walk_fn_c128_lo(int n, bool kahan)
{
    return kahan ? walk_fn_range<V_C128, true, 1>(n, std::make_integer_sequence<int, 24>{})
                 : walk_fn_range<V_C128, false, 1>(n, std::make_integer_sequence<int, 24>{});
}

}  // namespace permk
