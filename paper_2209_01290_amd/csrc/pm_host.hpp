// Host helpers shared by the C-ABI sources (defined in pm_capi.cpp).
#pragma once
#include <stdint.h>

#include <string>

#include "pm_internal.hpp"

namespace pm {

// Barrett constants of Alg. 4 for modulus q on 64-bit words (2 <= q < 2^62)
// and on 32-bit words (q odd, 3 <= q < 2^30); false if q is out of range.
bool make_mod(uint64_t q, Mod* M);
bool make_mod32(uint32_t q, Mod32* M);
// Which instantiation a modulus needs (KIND_WIDE or KIND_ANY).
int mod_kind(const Mod& M);
int mod_kind32(const Mod32& M);
// Records msg as the calling thread's last error and returns code.
int set_error(int code, const std::string& msg);

}  // namespace pm
