// Row pass for C = 2^4.
#define PM_LOGC 4
#include "row_kernel.inc"
