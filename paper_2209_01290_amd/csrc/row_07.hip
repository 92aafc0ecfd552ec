// Row pass for C = 2^7.
#define PM_LOGC 7
#include "row_kernel.inc"
