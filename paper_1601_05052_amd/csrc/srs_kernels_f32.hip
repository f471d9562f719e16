// Kernel instantiations for float input.
#define DD_TIN float
#define DD_TIN_NAME(prefix) prefix##f32
#include "srs_inst.inc"
