// Global-memory views of device pointers (kernel sources only).
//
// Pointers that a kernel reads out of an argument struct are generic to the
// compiler, so the loads and stores through them become FLAT instructions.
// A FLAT access counts against both the vector-memory and the LDS wait
// counters, so every LDS read after it waits for all outstanding FLAT loads
// and a register ring of prefetched rows no longer overlaps the products.
// Every pointer these helpers take points to global memory (hipMalloc'ed
// buffers or the library's own device arrays); the cast tells the compiler
// so, and the accesses become GLOBAL instructions.
#pragma once

#include <hip/hip_runtime.h>

namespace lrc {

template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Whole-object load and store through a global view, for types (such as the
// HIP vector types) whose member operators take generic references.
template <class V>
__device__ __forceinline__ V gload(const V* p) {
  V v;
  __builtin_memcpy(&v, gmem(p), sizeof(V));
  return v;
}
template <class V>
__device__ __forceinline__ void gstore(V* p, const V& v) {
  __builtin_memcpy(gmem(p), &v, sizeof(V));
}

}  // namespace lrc
