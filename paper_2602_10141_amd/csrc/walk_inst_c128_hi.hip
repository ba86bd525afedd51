// Instantiations of the Gray walk kernel (walk_impl.h): c128 hi.
#include "walk_impl.h"

namespace permk {

WalkFn walk_fn_c128_hi(int n, bool kahan)
{
    return kahan ? walk_fn_range<V_C128, true, 25>(n, std::make_integer_sequence<int, NMAX - 24>{})
                 : walk_fn_range<V_C128, false, 25>(n, std::make_integer_sequence<int, NMAX - 24>{});
}

}  // namespace permk
