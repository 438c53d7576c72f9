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

// A segment's view of a store: every array's address at the segment's
// first slot, uniform over a workgroup.  The loads and stores below take a
// 32-bit byte offset from it, so an access is a scalar base plus one 32-bit
// vector offset instead of a 64-bit address per array and lane.  Offsets
// are slots inside one segment (a few thousand, far below 2^29).
struct SegStore {
    SDMD_GLOBAL char *pos[3], *cell, *u[3], *w, *id;
};

template <class T>
__device__ __forceinline__ SegStore seg_store(const Store &s, long long first)
{
    using R = typename T::real;
    auto at = [&](void *q, long long size) -> SDMD_GLOBAL char * {
        return q ? gp((char *)q + first * size) : nullptr;
    };
    SegStore v;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        v.pos[a] = at(s.pos[a], sizeof(R));
        v.u[a] = at(s.u[a], sizeof(R));
    }
    v.cell = at(s.cell, sizeof(uint16_t));
    v.w = at(s.w, sizeof(R));
    v.id = at(s.id, sizeof(uint32_t));
    return v;
}

template <int DIM, class T>
__device__ __forceinline__ void load_part(const SegStore &v, uint32_t i, Part<T> &p)
{
    using R = typename T::real;
    const uint32_t o = i * (uint32_t)sizeof(R);
#pragma unroll
    for (int a = 0; a < DIM; ++a) p.pos[a] = *(const SDMD_GLOBAL R *)(v.pos[a] + o);
    if constexpr (T::split) p.cell = *(const SDMD_GLOBAL uint16_t *)(v.cell + i * 2u);
#pragma unroll
    for (int a = 0; a < 3; ++a) p.u[a] = *(const SDMD_GLOBAL R *)(v.u[a] + o);
    p.w = *(const SDMD_GLOBAL R *)(v.w + o);
    if (v.id) p.id = *(const SDMD_GLOBAL uint32_t *)(v.id + i * 4u);
}

template <int DIM, class T>
__device__ __forceinline__ void store_part(const SegStore &v, uint32_t i, const Part<T> &p, bool full)
{
    using R = typename T::real;
    const uint32_t o = i * (uint32_t)sizeof(R);
#pragma unroll
    for (int a = 0; a < DIM; ++a) *(SDMD_GLOBAL R *)(v.pos[a] + o) = p.pos[a];
    if constexpr (T::split) *(SDMD_GLOBAL uint16_t *)(v.cell + i * 2u) = (uint16_t)p.cell;
#pragma unroll
    for (int a = 0; a < 3; ++a) *(SDMD_GLOBAL R *)(v.u[a] + o) = p.u[a];
    if (full) {
        *(SDMD_GLOBAL R *)(v.w + o) = p.w;
        if (v.id) *(SDMD_GLOBAL uint32_t *)(v.id + i * 4u) = p.id;
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
