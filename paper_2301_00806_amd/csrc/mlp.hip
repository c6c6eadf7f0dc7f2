// Cost-model kernels (filled in with the learned scheduler).
#include <hip/hip_runtime.h>
