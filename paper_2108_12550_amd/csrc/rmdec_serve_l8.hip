// Serving kernel for list size 8 (codes of kServeCodes).
#include "rmdec_serve.hpp"

namespace rmdec {
// two waves per SIMD: the list-size-8 decoders need up to 256 VGPRs
ServeGroup serve_group_l8() { return ServeKernel<2, 8>::group(); }
} // namespace rmdec
