// Kernel instantiations for uint8_t input.
#define DD_TIN uint8_t
#define DD_TIN_NAME(prefix) prefix##u8
#include "srs_inst.inc"
