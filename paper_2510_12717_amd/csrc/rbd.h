// Rigid-body dynamics of a kinematic tree on the GPU (the real-time
// iteration's front and back end): the model as the kernels read it and the
// launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mpc_internal.h"

namespace mpc {

constexpr int kMaxBodies = 24;  // one degree of freedom per body (the humanoid's 6 + 18)
constexpr int kMaxU = 32;       // joint torques + foot wrenches

// Device copy of a model (arrays in device memory, one degree of freedom per
// body, bodies in topological order).
struct ModelDev {
  int n, n_feet, foot_dim;
  double gravity;
  const int32_t* parent;     // [n], -1 for the first body
  const int32_t* jtype;      // [n], 0 revolute, 1 prismatic
  const double* axis;        // [n][3], joint frame
  const double* offset;      // [n][3], joint frame origin in the parent frame
  const double* mass;        // [n]
  const double* com;         // [n][3], body frame
  const double* inertia;     // [n][3], principal, about the centre of mass
  const double* armature;    // [n], added to the mass matrix's diagonal
  const int32_t* foot_body;  // [n_feet]
  const double* foot_offset; // [n_feet][3], body frame
};

hipError_t launch_rnea(const ModelDev& md, int count, const double* q, const double* qd,
                       const double* qdd, const double* F, double* tau, hipStream_t s);
template <typename T>
hipError_t launch_linearize(const ModelDev& md, int n_agents, int N, double dt, const T* X, const T* U,
                            T* A, T* B, T* C, T* Jf, int32_t* status, hipStream_t s);
template <typename T>
hipError_t launch_rti_torque(const ModelDev& md, int count, int N, double dt, double kp, double kd,
                             const T* X, const T* U, const T* xm, T* tau, hipStream_t s);

}  // namespace mpc
