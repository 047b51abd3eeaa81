// tpm_dispatch.cpp -- element-type dispatch of the thread-per-matrix kernels.
#include <cstdlib>
#include <cstring>

#include "ci_launch.hpp"

namespace ci {

namespace {
int g_variant = -1;
}

int tpm_default_variant()
{
    if (g_variant < 0) {
        const char* e = std::getenv("CHOLINV_TPM_VARIANT");
        g_variant = VARIANT_AUTO;
        if (e && std::strcmp(e, "direct") == 0) g_variant = VARIANT_DIRECT;
        if (e && std::strcmp(e, "staged") == 0) g_variant = VARIANT_STAGED;
        if (e && std::strcmp(e, "persist") == 0) g_variant = VARIANT_PERSIST;
    }
    return g_variant;
}

void tpm_set_default_variant(int v) { g_variant = v; }

namespace {
int g_ns_engine = -1;
}

int ns_engine()
{
    if (g_ns_engine < 0) {
        const char* e = std::getenv("CHOLINV_NS_ENGINE");
        g_ns_engine = (e && std::strcmp(e, "lanes") == 0) ? NS_ENGINE_LANES : NS_ENGINE_MFMA;
    }
    return g_ns_engine;
}

int device_cus()
{
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0)
            n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

int tpm_nmax(int dtype, int mixed)
{
    switch (dtype) {
    case DT_F32: return mixed ? 8 : 16;
    case DT_F64: return 12;
    case DT_C64: return 8;
    case DT_C128: return 8;
    default: return 0;
    }
}

hipError_t launch_tpm(int dtype, int n, int op, int method, int mixed, const BatchArgs& p,
                      hipStream_t s)
{
    switch (dtype) {
    case DT_F32: return launch_tpm_f32(n, op, method, mixed, p, s);
    case DT_F64: return launch_tpm_f64(n, op, method, mixed, p, s);
    case DT_C64: return launch_tpm_c64(n, op, method, mixed, p, s);
    case DT_C128: return launch_tpm_c128(n, op, method, mixed, p, s);
    default: return hipErrorNotSupported;
    }
}

}  // namespace ci

namespace ci {

hipError_t launch_group(int dtype, int n, int op, int method, int mixed, const BatchArgs& p,
                        hipStream_t s)
{
    switch (dtype) {
    case DT_F32: return launch_group_f32(n, op, method, mixed, p, s);
    case DT_F64: return launch_group_f64(n, op, method, mixed, p, s);
    case DT_C64: return launch_group_c64(n, op, method, mixed, p, s);
    case DT_C128: return launch_group_c128(n, op, method, mixed, p, s);
    default: return hipErrorNotSupported;
    }
}

}  // namespace ci
