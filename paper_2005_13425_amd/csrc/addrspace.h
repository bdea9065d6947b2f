// Address-space-qualified pointers for kernel bodies that also run from a
// slot table.  A pointer read from memory has no known address space, so
// accesses through it compile to flat instructions (which also count against
// the LDS wait counter) and uniform loads lose their scalar form.  Kernel
// bodies therefore take
//   gptr<T>: device global memory (vector global loads, stores and atomics);
//   kptr<T>: device memory that no thread writes during the launch, read with
//            uniform addresses (scalar loads through the constant cache).
#pragma once

namespace nek {

#if defined(__HIP_DEVICE_COMPILE__)
template <typename T> using gptr = __attribute__((address_space(1))) T *;
template <typename T> using kptr = __attribute__((address_space(4))) const T *;
#else
// the host pass of a HIP source parses device bodies but never runs them; on
// the host target these address spaces mean nothing, so plain pointers
template <typename T> using gptr = T *;
template <typename T> using kptr = const T *;
#endif

}  // namespace nek
