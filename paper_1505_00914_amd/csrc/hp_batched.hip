// hp_batched.hip -- batched entry points (placeholder until the batched
// kernels land).
#include "hp_host.h"
