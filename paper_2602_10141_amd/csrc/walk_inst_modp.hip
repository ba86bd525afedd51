// Instantiations of the Gray walk kernel (walk_impl.h): modp.
#include "walk_impl.h"

namespace permk {

WalkFn walk_fn_modp(int n)
{
    return walk_fn_range<V_MODP, false, 1>(n, std::make_integer_sequence<int, NMAX>{});
}

}  // namespace permk
