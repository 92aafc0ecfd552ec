// Row pass for C = 2^10.
#define PM_LOGC 10
#include "row_kernel.inc"
