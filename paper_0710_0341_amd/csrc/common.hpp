// Shared device/host helpers for the osa library (gfx950, HIP).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>

#include "../../include/osa.h"

namespace osa {

// ---------------------------------------------------------------- complex
typedef double2 cd;   // complex128 (re, im)
typedef float2 cf;    // complex64

__host__ __device__ __forceinline__ cd mk(double r, double i) { return make_double2(r, i); }
__host__ __device__ __forceinline__ cd cadd(cd a, cd b) { return mk(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ cd csub(cd a, cd b) { return mk(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ cd cmul(cd a, cd b) {
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ __forceinline__ cd cmulc(cd a, cd b) {
    return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ __forceinline__ cd cscale(cd a, double s) { return mk(a.x * s, a.y * s); }
__host__ __device__ __forceinline__ cd cconj(cd a) { return mk(a.x, -a.y); }
__host__ __device__ __forceinline__ double cabs2(cd a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ __forceinline__ double cabsd(cd a) { return sqrt(a.x * a.x + a.y * a.y); }
__host__ __device__ __forceinline__ cd cdiv(cd a, cd b) {
    // Smith's algorithm avoids overflow for badly scaled operands.
    if (fabs(b.x) >= fabs(b.y)) {
        double r = b.y / b.x, d = b.x + b.y * r;
        return mk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
    } else {
        double r = b.x / b.y, d = b.x * r + b.y;
        return mk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
    }
}
__host__ __device__ __forceinline__ cd cinv(cd b) { return cdiv(mk(1.0, 0.0), b); }
// a += b * c
__host__ __device__ __forceinline__ void cfma(cd& a, cd b, cd c) {
    a.x = fma(b.x, c.x, a.x); a.x = fma(-b.y, c.y, a.x);
    a.y = fma(b.x, c.y, a.y); a.y = fma(b.y, c.x, a.y);
}
// a += conj(b) * c
__host__ __device__ __forceinline__ void cfmac(cd& a, cd b, cd c) {
    a.x = fma(b.x, c.x, a.x); a.x = fma(b.y, c.y, a.x);
    a.y = fma(b.x, c.y, a.y); a.y = fma(-b.y, c.x, a.y);
}

// conversions between storage types and the double accumulator
__host__ __device__ __forceinline__ cd tod(cd a) { return a; }
__host__ __device__ __forceinline__ cd tod(cf a) { return mk((double)a.x, (double)a.y); }
template <typename T> __host__ __device__ __forceinline__ T fromd(cd a);
template <> __host__ __device__ __forceinline__ cd fromd<cd>(cd a) { return a; }
template <> __host__ __device__ __forceinline__ cf fromd<cf>(cd a) {
    return make_float2((float)a.x, (float)a.y);
}

// ---------------------------------------------------------------- geometry
struct Geom {
    int lx, ly, lz, lt;   // extents
    int V;                // sites
    int Vp;               // padded sites (multiple of 64); component stride of a vector
    int apt;              // antiperiodic time boundary
    int64_t N() const { return 12LL * Vp; }   // internal vector length (complex entries)
};

// ---------------------------------------------------------------- errors
struct HipError { hipError_t e; const char* where; };

#define OSA_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) throw ::osa::HipError{e_, #call};                    \
    } while (0)

#define OSA_LAUNCH_CHECK() OSA_HIP(hipGetLastError())

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace osa
