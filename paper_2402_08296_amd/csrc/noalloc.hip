// Scratch memory of the allocation-free entry points: a file-scope device
// array instead of device memory allocated by the library. Each device the
// library runs on holds its own copy until the process ends; its address on
// a device is looked up once, with that device current, when the first
// context of the device is created, and only that address is handed to
// kernels and copies (the array's name is a host-side stand-in in host code).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "device.h"

namespace ddmgnn {

namespace {
// The dot product's per-workgroup partial sums (one problem's vector grid).
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

std::mutex g_mu;
std::map<int, double*> g_ptr;  // device -> address of its copy of scratch
}  // namespace

hipError_t noalloc_init(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr.count(device)) return hipSuccess;
    double* p = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
    return hipSuccess;
}

double* noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    const auto it = g_ptr.find(device);
    return it == g_ptr.end() ? nullptr : it->second;
}

}  // namespace ddmgnn
