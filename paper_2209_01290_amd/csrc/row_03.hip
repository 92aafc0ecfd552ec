// Row pass for C = 2^3.
#define PM_LOGC 3
#include "row_kernel.inc"
