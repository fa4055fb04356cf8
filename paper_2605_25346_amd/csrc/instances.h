// Kernel handles of the chain-kernel instance sets (one translation unit per chain type
// and tile count, see instances.hip).
#pragma once

enum {
  DR_KIND_BOUND = 0,   // k_bound_init (variant bit 0: weights staged in LDS; bit 1: row tiles in pairs)
  DR_KIND_FINAL = 1,   // k_final, plain spec rows
  DR_KIND_DUAL = 2,    // k_final, dual ascent (variant 1: per-item LDS copy of the relaxation)
  DR_KIND_REACH = 3,   // k_reach_dt
  DR_KIND_PGRAD = 4,   // k_final, dual adjoint with parameter-gradient tapes (variant 1: item copy)
  DR_KIND_JOINT = 5,   // k_reach_joint (CROWN through the unrolled closed loop)
  DR_KIND_RGRAD = 6,   // k_reach_grad (reverse pass through the stepwise reach)
  DR_KIND_CT = 7       // k_ct_control (controller step of the continuous-time closed loop)
};

#define DR_DECLARE_INSTANCE(T, NT) const void* dr_instance_##T##_##NT(int kind, int variant);
DR_DECLARE_INSTANCE(float, 2)
DR_DECLARE_INSTANCE(float, 4)
DR_DECLARE_INSTANCE(float, 6)
DR_DECLARE_INSTANCE(float, 8)
DR_DECLARE_INSTANCE(float, 16)
DR_DECLARE_INSTANCE(double, 2)
DR_DECLARE_INSTANCE(double, 4)
DR_DECLARE_INSTANCE(double, 6)
DR_DECLARE_INSTANCE(double, 8)
DR_DECLARE_INSTANCE(double, 16)
#undef DR_DECLARE_INSTANCE
