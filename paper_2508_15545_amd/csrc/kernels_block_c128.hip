// The register-block kernels for complex128 states (one translation unit per
// element type, compiled in parallel with the other).
#define QV_BLOCK_ELEM 16
#include "kernels_block.hip"
