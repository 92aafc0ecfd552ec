// Row pass for C = 2^2.
#define PM_LOGC 2
#include "row_kernel.inc"
