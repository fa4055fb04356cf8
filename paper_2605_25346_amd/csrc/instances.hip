// One instance set of the chain kernels: chain type DR_T (float or double) and DR_NT
// 16-tiles per hidden layer, selected on the compiler line.  Each set is its own
// translation unit so that the sets compile in parallel; the host side reaches the
// kernels through the function below (kernel handles are valid across translation
// units of one shared library).
#include "bound_kernels.hpp"
#include "joint_kernels.hpp"
#include "grad_kernels.hpp"
#include "ct_kernels.hpp"
#include "instances.h"

#ifndef DR_T
#error "DR_T (float or double) must be defined"
#endif
#ifndef DR_NT
#error "DR_NT (2, 4, 6, 8 or 16) must be defined"
#endif

#define DR_CAT2(a, b, c) a##b##_##c
#define DR_CAT(a, b, c) DR_CAT2(a, b, c)

const void* DR_CAT(dr_instance_, DR_T, DR_NT)(int kind, int variant) {
  using T = DR_T;
  constexpr int NT = DR_NT;
  switch (kind) {
    case DR_KIND_BOUND:
      // narrow networks run one subdomain per wavefront (variant bit 0: weights staged in
      // LDS; bit 1: FP32 row tiles in pairs); wider ones one subdomain per workgroup
      if constexpr (NT <= 4) {
        constexpr int NR2 = sizeof(T) == 4 ? 2 : 1;
        switch (variant) {
          case 0: return (const void*)&dr::k_bound_init<T, NT, false, 64, 1>;
          case 1: return (const void*)&dr::k_bound_init<T, NT, true, 64, 1>;
          case 2: return (const void*)&dr::k_bound_init<T, NT, false, 64, NR2>;
          case 3: return (const void*)&dr::k_bound_init<T, NT, true, 64, NR2>;
          default: return nullptr;
        }
      } else {
        return variant ? nullptr : (const void*)&dr::k_bound_init<T, NT, false, 256>;
      }
    case DR_KIND_FINAL: return (const void*)&dr::k_final<T, NT, false>;
    case DR_KIND_DUAL:
      return variant ? (const void*)&dr::k_final<T, NT, true, true> : (const void*)&dr::k_final<T, NT, true>;
    case DR_KIND_REACH: return (const void*)&dr::k_reach_dt<T, NT>;
    case DR_KIND_PGRAD:
      return variant ? (const void*)&dr::k_final<T, NT, true, true, true> : (const void*)&dr::k_final<T, NT, true, false, true>;
    case DR_KIND_JOINT: return variant ? nullptr : (const void*)&dr::k_reach_joint<T, NT>;
    case DR_KIND_RGRAD: return variant ? nullptr : (const void*)&dr::k_reach_grad<T, NT>;
    case DR_KIND_CT: return variant ? nullptr : (const void*)&dr::k_ct_control<T, NT>;
    default: return nullptr;
  }
}
