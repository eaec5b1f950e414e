// Serving kernel for list size 1 (codes of kServeCodes).
#include "rmdec_serve.hpp"

namespace rmdec {
ServeGroup serve_group_l1() { return ServeKernel<3, 1>::group(); }
} // namespace rmdec
