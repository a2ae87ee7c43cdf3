// Shape dispatch and LDS sizing shared by the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_ntt.hpp"

namespace ephdc {

using namespace ephdc_dev;

// Dynamic LDS of every kernel of a shape (exchange buffers and, if it fits, the table).
template <int LOGN, int LE>
inline size_t lds_bytes() {
  return sizeof(uint32_t) * LdsPlan<LOGN, LE>::words;
}

// Dynamic LDS of the kernels that run one transform per workgroup without the table and
// take the single-buffer exchanges where one_buffer() holds.
template <int LOGN, int LE>
inline size_t lds_bytes_one_transform() {
  return one_buffer<LOGN, LE>() ? sizeof(uint32_t) * Shape<LOGN, LE>::PADN : lds_bytes<LOGN, LE>();
}

// Calls f with the compile-time shape (LOGN, LE) of a supported ring degree; `le` selects
// the values per thread (0: the default of the degree).
template <class F>
inline hipError_t dispatch(int logn, int le, F&& f) {
  using std::integral_constant;
  switch (logn * 16 + le) {
    case 11 * 16 + 0:
    case 11 * 16 + 3: return f(integral_constant<int, 11>{}, integral_constant<int, 3>{});
    case 12 * 16 + 0:
    case 12 * 16 + 3: return f(integral_constant<int, 12>{}, integral_constant<int, 3>{});
    case 13 * 16 + 3: return f(integral_constant<int, 13>{}, integral_constant<int, 3>{});
    case 13 * 16 + 0:
    case 13 * 16 + 4: return f(integral_constant<int, 13>{}, integral_constant<int, 4>{});
    case 14 * 16 + 0:
    case 14 * 16 + 4: return f(integral_constant<int, 14>{}, integral_constant<int, 4>{});
    case 14 * 16 + 5: return f(integral_constant<int, 14>{}, integral_constant<int, 5>{});
    default: return hipErrorInvalidValue;
  }
}

template <class F>
inline hipError_t dispatch(int logn, F&& f) {
  return dispatch(logn, 0, f);
}


hipError_t prepare_ks_kernels();

}  // namespace ephdc
