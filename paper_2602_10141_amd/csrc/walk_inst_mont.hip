// Instantiations of the Gray walk kernel (walk_impl.h): mont.
#include "walk_impl.h"

namespace permk {

WalkFn walk_fn_mont(int n)
{
    return walk_fn_range<V_MONT, false, 1>(n, std::make_integer_sequence<int, NMAX>{});
}

}  // namespace permk
