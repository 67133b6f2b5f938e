// Host-side helpers shared by the translation units of libwcnst.
#pragma once

#include <hip/hip_runtime.h>

#include <stddef.h>

#include "wcnst.h"

// Records a thread-local message (read by wcnst_last_error) and returns st.
wcnst_status wcnst_fail(wcnst_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
wcnst_status wcnst_check_desc(const wcnst_desc* d);
int wcnst_desc_nvar(const wcnst_desc* d);
size_t wcnst_align256(size_t b);

#define WCNST_HIP_TRY(expr)                                                                \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return wcnst_fail(WCNST_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)
