// The register-block kernels for complex64 states (one translation unit per
// element type, compiled in parallel with the other).
#define QV_BLOCK_ELEM 8
#include "kernels_block.hip"
