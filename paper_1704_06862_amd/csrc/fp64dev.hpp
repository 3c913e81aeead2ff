// FP64 vector and complex helpers for the device-side set-up kernels
// (near-field fill, ILU(0) factorisation).
#pragma once

#include <hip/hip_runtime.h>

namespace sfmm {
namespace fp64 {

struct d3 {
    double x, y, z;
};
__device__ inline d3 operator+(d3 a, d3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline d3 operator-(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline d3 operator*(double s, d3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline double dotp(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline d3 crossp(d3 a, d3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
__device__ inline double normp(d3 a) { return sqrt(dotp(a, a)); }

struct zc {
    double r, i;
};
__device__ inline zc operator+(zc a, zc b) { return {a.r + b.r, a.i + b.i}; }
__device__ inline zc operator-(zc a, zc b) { return {a.r - b.r, a.i - b.i}; }
__device__ inline zc operator*(zc a, zc b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ inline zc operator*(double s, zc a) { return {s * a.r, s * a.i}; }
__device__ inline zc operator*(zc a, double s) { return {s * a.r, s * a.i}; }
__device__ inline zc zdiv(zc a, zc b) {
    const double d = b.r * b.r + b.i * b.i;
    return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}
// complex vector (three components)
struct zv {
    zc x, y, z;
};
__device__ inline zc zdot(d3 a, const zv &v) { return a.x * v.x + a.y * v.y + a.z * v.z; }


}  // namespace fp64
}  // namespace sfmm
