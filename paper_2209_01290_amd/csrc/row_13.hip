// Row pass for C = 2^13.
#define PM_LOGC 13
#include "row_kernel.inc"
