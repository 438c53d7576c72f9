// part.h -- one macro-particle in registers and its SoA load / store.
#pragma once

#include "sdmd_dev.h"

namespace sdmd {

template <class T>
struct Part {
    using R = typename T::real;
    R pos[3];
    int cell;
    R u[3];
    R w;
    uint32_t id;
};

template <int DIM, class T>
__device__ __forceinline__ void load_part(const Store &s, long long i, Part<T> &p)
{
    using R = typename T::real;
#pragma unroll
    for (int a = 0; a < DIM; ++a) p.pos[a] = gp((const R *)s.pos[a])[i];
    if constexpr (T::split) p.cell = gp((const uint16_t *)s.cell)[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) p.u[a] = gp((const R *)s.u[a])[i];
    p.w = gp((const R *)s.w)[i];
    if (s.id) p.id = gp((const uint32_t *)s.id)[i];
}

template <int DIM, class T>
__device__ __forceinline__ void store_part(const Store &s, long long i, const Part<T> &p, bool full)
{
    using R = typename T::real;
#pragma unroll
    for (int a = 0; a < DIM; ++a) gp((R *)s.pos[a])[i] = p.pos[a];
    if constexpr (T::split) gp(s.cell)[i] = (uint16_t)p.cell;
#pragma unroll
    for (int a = 0; a < 3; ++a) gp((R *)s.u[a])[i] = p.u[a];
    if (full) {
        gp((R *)s.w)[i] = p.w;
        if (s.id) gp(s.id)[i] = p.id;
    }
}

template <int DIM, class T>
__device__ __forceinline__ void copy_part(const Store &from, long long i, const Store &to, long long j)
{
    Part<T> p;
    load_part<DIM, T>(from, i, p);
    store_part<DIM, T>(to, j, p, true);
}

}  // namespace sdmd
