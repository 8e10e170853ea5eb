// Device-side helpers shared by the level kernels (cos_level.hip) and the
// sublattice level kernels (cos_sub.hip).
#pragma once
#include "cos_internal.hpp"

namespace libcos {

#define COS_RF(x) __builtin_amdgcn_readfirstlane(x)

typedef __attribute__((address_space(3))) double lds_double;
// read-only tables read at wave-uniform addresses: through the constant
// address space they are fetched with scalar loads
typedef const __attribute__((address_space(4))) int32_t cint32;

__device__ __forceinline__ int4 load_level(const DevPlan &P, int l) {
    const cint32 *p = (const cint32 *)(P.levels + l);
    return make_int4(p[0], p[1], p[2], p[3]);
}

// LDS byte address of a __shared__ pointer
__device__ __forceinline__ uint32_t lds_addr(double *p) {
    return (uint32_t)(uintptr_t)(lds_double *)p;
}

// a lane's word of a 64-wide slot: wave-uniform base + the lane's byte offset
// (scalar base registers, one 32-bit offset register per lane)
// (the empty asm pins the base in scalar registers, so that it is not folded
// into a per-lane 64-bit address)
typedef __attribute__((address_space(1))) char global_char;
__device__ __forceinline__ double lane_ld(const double *base, uint32_t lane8) {
    const global_char *p = (const global_char *)base;
    asm volatile("" : "+s"(p));
    return *(const __attribute__((address_space(1))) double *)(p + lane8);
}
// the same with the nontemporal hint, for DP states: a level writes or reads
// each state once, and a level's states are far larger than the caches, so
// they stream past them instead of evicting the tables and matrices
__device__ __forceinline__ double lane_ld_nt(const double *base, uint32_t lane8) {
    const global_char *p = (const global_char *)base;
    asm volatile("" : "+s"(p));
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) double *)(p + lane8));
}
__device__ __forceinline__ void lane_st_nt(double *base, uint32_t lane8, double x) {
    global_char *p = (global_char *)base;
    asm volatile("" : "+s"(p));
    __builtin_nontemporal_store(x, (__attribute__((address_space(1))) double *)(p + lane8));
}
__device__ __forceinline__ void lane_st(double *base, uint32_t lane8, double x) {
    global_char *p = (global_char *)base;
    asm volatile("" : "+s"(p));
    *(__attribute__((address_space(1))) double *)(p + lane8) = x;
}

}  // namespace libcos
