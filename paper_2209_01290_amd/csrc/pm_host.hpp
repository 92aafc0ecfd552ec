// Host helpers shared by the C-ABI sources (defined in pm_capi.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
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

// PM_VALIDATE (environment): when set and not "0", entry points also check
// their inputs' preconditions on the device (synchronising the stream).
bool validate_enabled();
// Every word of x[l*per_limb .. (l+1)*per_limb) is < q[l], for l < limbs
// (word_bytes 8 or 4); PM_OK or PM_EINVAL naming `name`.
int validate_canonical(const void* x, int word_bytes, size_t per_limb, size_t limbs, const uint64_t* q,
                       const std::string& name, hipStream_t s);
// psi = tw[l*N + N/2] satisfies psi^N = q[l] - 1 for every limb l.
int validate_psi(const void* tw, int word_bytes, size_t N, size_t limbs, const uint64_t* q, const std::string& name,
                 hipStream_t s);

}  // namespace pm
