// Serving kernel for list size 4 (codes of kServeCodes).
#include "rmdec_serve.hpp"

namespace rmdec {
ServeGroup serve_group_l4() { return ServeKernel<3, 4>::group(); }
} // namespace rmdec
