// Row pass for C = 2^6.
#define PM_LOGC 6
#include "row_kernel.inc"
