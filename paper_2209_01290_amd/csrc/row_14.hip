// Row pass for C = 2^14.
#define PM_LOGC 14
#include "row_kernel.inc"
