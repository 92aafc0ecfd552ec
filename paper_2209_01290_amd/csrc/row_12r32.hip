// Product rows of 2^12 words with the split's radix fixed at compile time,
// 32-bit words, any modulus they take (both reductions of modarith32.hpp).
#include "row_fixed.inc"

namespace pm {

bool launch_row12_fixed(int kind, int mode, const RowArgsT<uint32_t>& a, hipStream_t s) {
  return kind == KIND_WIDE ? launch_kind<uint32_t, KIND_WIDE>(mode, a, s)
                           : launch_kind<uint32_t, KIND_ANY>(mode, a, s);
}

}  // namespace pm
