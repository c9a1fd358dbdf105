// stubs.hip -- entry points not yet implemented (return FTK_ERR_ARG with a message).
#include <hip/hip_runtime.h>

#include "../../include/ftk.h"

extern "C" {
}
