// Row pass for C = 2^9.
#define PM_LOGC 9
#include "row_kernel.inc"
