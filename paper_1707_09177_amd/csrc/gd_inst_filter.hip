// filter_apply kernels for both dtypes and every single-shape tile variant.
#include "gd_kernels.h"

namespace gd {

template <typename T>
static const void *filter_ptr(int variant) {
    constexpr int VM = VMax<T>::v;
#define GD_F(v) \
    case v: return reinterpret_cast<const void *>(&filter_kernel<T, v>)
    switch (variant) {
        GD_F(var_code(2, VM, 1));
        GD_F(var_code(2, 1, 1));
        GD_F(var_code(3, VM, 1));
        GD_F(var_code(3, VM, 2));
        GD_F(var_code(3, 1, 4));
        GD_F(var_code(3, 1, 1));
    default: return nullptr;
    }
#undef GD_F
}

const void *filter_kernel_ptr(int dtype, int variant) {
    return dtype == GD_F32 ? filter_ptr<float>(variant) : filter_ptr<double>(variant);
}

}  // namespace gd
