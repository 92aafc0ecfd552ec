// Row pass for C = 2^5.
#define PM_LOGC 5
#include "row_kernel.inc"
