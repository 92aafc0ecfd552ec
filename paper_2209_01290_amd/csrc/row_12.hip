// Row pass for C = 2^12.
#define PM_LOGC 12
#include "row_kernel.inc"
