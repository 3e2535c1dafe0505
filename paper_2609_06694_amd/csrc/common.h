// Device-side helpers shared by the stencil kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stk {

constexpr int kStar = 0;
constexpr int kBox = 1;
constexpr int kPeriodic = 0;
constexpr int kZero = 1;
constexpr int kThreads = 256;      // every kernel runs 4 waves of 64
constexpr int kWave = 64;
constexpr int kXcds = 8;           // MI355X: 8 accelerator dies, 32 CUs each
constexpr int kMaxTaps = 125;      // 3D box r = 2
constexpr int kMaxRadius = 4;

// Compact coefficient list, passed by value as a kernel argument.
//  box : dense (dz, dy, dx) lexicographic order, dx fastest
//  star: [centre, x:-r..-1,+1..+r, y:-r..-1,+1..+r, z:-r..-1,+1..+r]
struct Taps {
    float c[kMaxTaps];
    float sum;   // sum of all weights (for the difference form of a star)
};

template <int R>
__host__ __device__ constexpr int star_x(int d) { return d < 0 ? 1 + (d + R) : R + d; }
template <int R>
__host__ __device__ constexpr int star_y(int d) { return 2 * R + (d < 0 ? 1 + (d + R) : R + d); }
template <int R>
__host__ __device__ constexpr int star_z(int d) { return 4 * R + (d < 0 ? 1 + (d + R) : R + d); }
template <int R>
__host__ __device__ constexpr int box2(int dy, int dx) { return (dy + R) * (2 * R + 1) + (dx + R); }
template <int R>
__host__ __device__ constexpr int box3(int dz, int dy, int dx) {
    return ((dz + R) * (2 * R + 1) + (dy + R)) * (2 * R + 1) + (dx + R);
}

// Storage conversions.  fp16 is IEEE binary16; narrowing rounds to nearest even.
__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(_Float16 v) { return (float)v; }
template <typename T>
__device__ __forceinline__ T from_f32(float v);
template <>
__device__ __forceinline__ float from_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ _Float16 from_f32<_Float16>(float v) { return (_Float16)v; }
// Round a value to what the storage type can hold (identity for f32).
template <typename T>
__device__ __forceinline__ float round_to_storage(float v) { return to_f32(from_f32<T>(v)); }

// Arithmetic type of a storage type: f32 for fp16 and f32 storage, f64 for
// f64 storage.
template <typename T>
struct AccOf {
    using type = float;
};
template <>
struct AccOf<double> {
    using type = double;
};
template <typename T>
using acc_t = typename AccOf<T>::type;
__device__ __forceinline__ double to_f64(double v) { return v; }
// Stored value -> arithmetic type, and back (rounding to nearest even).
template <typename T>
__device__ __forceinline__ acc_t<T> to_acc(T v) {
    if constexpr (sizeof(acc_t<T>) == 8) return to_f64(v);
    else return to_f32(v);
}
template <typename T>
__device__ __forceinline__ T from_acc(acc_t<T> v) {
    if constexpr (sizeof(acc_t<T>) == 8) return v;
    else return from_f32<T>(v);
}
__device__ __forceinline__ float fma_acc(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_acc(double a, double b, double c) { return fma(a, b, c); }

// Workgroups are handed to the XCDs round-robin in launch order.  Renumber
// them so each XCD receives one contiguous run of logical tiles: neighbouring
// tiles then share halo rows through the same L2.  Bijective for any count.
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    const int xcd = b % kXcds, idx = b / kXcds;
    const int q = nblocks / kXcds, rem = nblocks % kXcds;
    return xcd * q + (xcd < rem ? xcd : rem) + idx;
}

__device__ __forceinline__ int wrap_index(int i, int n) {
    int m = i % n;
    return m < 0 ? m + n : m;
}

}  // namespace stk
