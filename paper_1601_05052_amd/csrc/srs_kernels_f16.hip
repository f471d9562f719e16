// Kernel instantiations for _Float16 input.
#define DD_TIN _Float16
#define DD_TIN_NAME(prefix) prefix##f16
#include "srs_inst.inc"
