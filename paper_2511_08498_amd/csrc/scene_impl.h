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

namespace rt {
// Sub-allocation of a caller-owned device workspace: pieces are taken in a
// fixed order, each rounded up to 256 bytes (so every piece is 256-byte
// aligned when the base is).  With a null base nothing is handed out and
// `used` is the size the same sequence needs (the size queries run it so).
struct Carver {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    template <typename T>
    bool take(T** p, size_t count)
    {
        const size_t nbytes = ((std::max<size_t>(count * sizeof(T), 1) + 255) / 256) * 256;
        if (base) {
            if (used + nbytes > cap) return false;
            *p = (T*)(base + used);
        } else {
            *p = nullptr;
        }
        used += nbytes;
        return true;
    }
};
}  // namespace rt

struct rt_scene {
    rt_scene_desc desc;
    rt::Geo g;
    rt::Inputs in;
    rt::SceneBufs b;
    int n_active = 0;
    std::vector<double> lam;
    std::vector<double> lam0;
    size_t bytes = 0;  // workspace bytes the scene uses (from the caller's d_ws)
    int batch_begin = -1, batch_end = -1;
    int storage = RT_F32;
    int cav_rec = 0;
    int cav_lp_dtype = -1;  // dtype currently encoded in b.cav_lp (-1: none)
    int cav_mode = -1;      // rt_avg the Core-and-Voigt chain was built with (-1: none)
};

namespace rt {
TraceLaunch make_trace(const rt_scene* sc, const rt_trace_params* p);
}  // namespace rt
