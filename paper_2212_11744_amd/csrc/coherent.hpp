// Data exchanged between the waves of one launch, and the status words that announce it.
//
// Access policies.  PlainAcc: ordinary loads and stores (LDS, data private to one wave, or data
// read only by later launches).  DevAcc: relaxed atomic loads and stores at agent scope, which are
// coherent per location across the XCDs of the device without any cache maintenance (they go past
// the non-coherent caches).  An agent-scope release or acquire would instead write back or
// invalidate a whole L2 on every use.
//
// Protocol: a producer writes its payload with DevAcc stores and then a status word with
// lq_flag_store, which first waits until every earlier store of the wave is complete at device
// scope; a consumer loads status words with lq_flag_load and, once the ones it needs are set,
// issues its DevAcc payload loads after lq_acquire.
#pragma once

#include <hip/hip_runtime.h>

namespace lqt {

struct PlainAcc {
  template <class R>
  static __device__ __forceinline__ void st(R* p, R v) { *p = v; }
  template <class R>
  static __device__ __forceinline__ R ld(const R* p) { return *p; }
};
struct DevAcc {
  template <class R>
  static __device__ __forceinline__ void st(R* p, R v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  template <class R>
  static __device__ __forceinline__ R ld(const R* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};

__device__ __forceinline__ unsigned lq_flag_load(const unsigned* f) { return DevAcc::ld(f); }

// Stores status word v once every earlier store of this wave is complete at device scope
// (s_waitcnt vmcnt(0) is a wave-wide wait; the compiler barriers keep the stores on their side).
__device__ __forceinline__ void lq_flag_store(unsigned* f, unsigned v) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt unconstrained (GFX9 encoding)
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  DevAcc::st(f, v);
}

// Payload loads of records whose status was just seen are issued after the status loads returned
// (their values decided the branch that leads here); the barrier keeps the compiler from moving
// them above.
__device__ __forceinline__ void lq_acquire() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

}  // namespace lqt
