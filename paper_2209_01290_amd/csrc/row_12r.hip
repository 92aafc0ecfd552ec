// Product rows of 2^12 words with the split's radix fixed at compile time,
// 64-bit words, moduli of 34..61 bits (KIND_WIDE: every 60-bit NTT prime).
#include "row_fixed.inc"

namespace pm {

bool launch_row12_fixed(int kind, int mode, const RowArgs& a, hipStream_t s) {
  return kind == KIND_WIDE && launch_kind<uint64_t, KIND_WIDE>(mode, a, s);
}

}  // namespace pm
