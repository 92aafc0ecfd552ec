// Row pass for C = 2^8.
#define PM_LOGC 8
#include "row_kernel.inc"
