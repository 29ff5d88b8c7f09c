// One instantiation unit of the counting kernel per pattern size k (built
// once per k with -DGP_INST_K=k), so the variants compile in parallel.
#include "count_kernel.hpp"

#ifndef GP_INST_K
#error "GP_INST_K must be defined"
#endif

namespace gpcount {

namespace {
template <int K, int G, int LEAF, int IEP = 0>
KernelFn pick_mode(int mode) {
    switch (mode) {
        case MODE_PLAIN: return count_kernel<K, G, LEAF, MODE_PLAIN, IEP>;
        case MODE_PER_ROOT: return count_kernel<K, G, LEAF, MODE_PER_ROOT, IEP>;
        case MODE_ACCOUNT: return count_kernel<K, G, LEAF, MODE_ACCOUNT, IEP>;
        default: return nullptr;
    }
}

template <int K, int G>
KernelFn pick_leaf(int leaf, int mode) {
    if (leaf == 2) return pick_mode<K, G, 2>(mode);
    if (leaf == 3 && K >= 5) return pick_mode<K, G, (K >= 5 ? 3 : 1)>(mode);
    if (leaf == 4 && K >= 4) return pick_mode<K, G, (K >= 4 ? 4 : 1)>(mode);
    return pick_mode<K, G, 1>(mode);
}

// IEP kernels, one per depth n (2 .. min(4, K - 2)); the leaf mode does not
// apply (the search stops at the last outer level)
template <int K, int G>
KernelFn pick_iep(int n, int mode) {
    if constexpr (K >= 4) {
        if (n == 2) return pick_mode<K, G, 1, 2>(mode);
    }
    if constexpr (K >= 5) {
        if (n == 3) return pick_mode<K, G, 1, 3>(mode);
    }
    if constexpr (K >= 6) {
        if (n == 4) return pick_mode<K, G, 1, 4>(mode);
    }
    return nullptr;
}
}  // namespace

#define GP_CAT2(a, b) a##b
#define GP_CAT(a, b) GP_CAT2(a, b)

KernelFn GP_CAT(pick_kernel_k, GP_INST_K)(int group, int leaf, int mode, int iep) {
    if (iep) return group == 64 ? pick_iep<GP_INST_K, 64>(iep, mode) : pick_iep<GP_INST_K, 32>(iep, mode);
    switch (group) {
        case 64: return pick_leaf<GP_INST_K, 64>(leaf, mode);
        case 32: return pick_leaf<GP_INST_K, 32>(leaf, mode);
        case 16: return pick_leaf<GP_INST_K, 16>(leaf, mode);
        case 8: return pick_leaf<GP_INST_K, 8>(leaf, mode);
        default: return nullptr;
    }
}

}  // namespace gpcount
