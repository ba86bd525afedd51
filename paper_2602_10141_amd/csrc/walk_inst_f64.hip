// Instantiations of the Gray walk kernel (walk_impl.h): f64.
#include "walk_impl.h"

namespace permk {

WalkFn walk_fn_f64(int n, bool kahan)
{
    return kahan ? walk_fn_range<V_F64, true, 1>(n, std::make_integer_sequence<int, NMAX>{})
                 : walk_fn_range<V_F64, false, 1>(n, std::make_integer_sequence<int, NMAX>{});
}

}  // namespace permk
