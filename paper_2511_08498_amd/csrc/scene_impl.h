// Scene handle internals shared by the host-side translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <vector>

#include "common.h"

namespace rt {
// Records a thread-local error message and returns st.
rt_status set_error(rt_status st, const char* fmt, ...);
}  // namespace rt

struct rt_scene {
    rt_scene_desc desc;
    rt::Geo g;
    rt::Inputs in;
    rt::SceneBufs b;
    int n_active = 0;
    std::vector<double> lam;
    std::vector<double> lam0;
    std::vector<void*> allocs;
    size_t bytes = 0;
    int batch_begin = -1, batch_end = -1;
    int storage = RT_F32;
    int cav_rec = 0;
    int cav_lp_dtype = -1;  // dtype currently encoded in b.cav_lp (-1: none)
    int cav_mode = -1;      // rt_avg the Core-and-Voigt chain was built with (-1: none)

    ~rt_scene()
    {
        for (void* p : allocs) (void)hipFree(p);
    }
    template <typename T>
    rt_status alloc(T** p, size_t count)
    {
        size_t nbytes = std::max<size_t>(count * sizeof(T), 256);
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, nbytes);
        if (e != hipSuccess) return rt::set_error(RT_E_HIP, "hipMalloc(%zu) failed: %s", nbytes, hipGetErrorString(e));
        allocs.push_back(q);
        bytes += nbytes;
        *p = (T*)q;
        return RT_OK;
    }
};


namespace rt {
TraceLaunch make_trace(const rt_scene* sc, const rt_trace_params* p);
}  // namespace rt
