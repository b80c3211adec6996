// Stream status: the one plain call that synchronises.
#include <hip/hip_runtime.h>

#include "adct.h"

extern "C" {

int adct_check(void* stream) {
    const hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    const hipError_t last = hipGetLastError();
    return e == hipSuccess && last == hipSuccess ? ADCT_OK : ADCT_E_HIP;
}

}  // extern "C"
