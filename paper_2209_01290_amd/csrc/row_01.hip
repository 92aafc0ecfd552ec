// Row pass for C = 2^1.
#define PM_LOGC 1
#include "row_kernel.inc"
