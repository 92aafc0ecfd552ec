// Row pass for C = 2^11.
#define PM_LOGC 11
#include "row_kernel.inc"
