// Host-side helpers shared by the C-ABI files (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <string>

#include "../../include/ppgmres.h"
#include "host_core.h"

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            ppg::set_error(std::string("HIP error ") + hipGetErrorString(e_) + " in " + #expr); \
            return PP_EDEVICE;                                                             \
        }                                                                                  \
    } while (0)

#define PP_TRY(expr)           \
    do {                       \
        pp_status s_ = (expr); \
        if (s_ < 0) return s_; \
    } while (0)

namespace ppg {

template <typename T>
inline pp_status dev_alloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) return PP_OK;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        set_error(std::string("hipMalloc failed: ") + hipGetErrorString(e));
        return PP_ENOMEM;
    }
    return PP_OK;
}

template <typename T>
inline void dev_free(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

inline hipStream_t S(void *s) { return (hipStream_t)s; }

inline double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace ppg
