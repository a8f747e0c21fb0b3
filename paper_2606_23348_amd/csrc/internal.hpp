// internal.hpp -- launch arguments and launchers shared by the host ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace gen {

struct EnvArgs {
    Geom g;
    GenParamsDev prm;
    uint64_t seed, env_base;
    EnvScalars *sc;
    int8_t *owner;
    uint8_t *type;
    int32_t *army;
    const int32_t *actions;
    uint8_t *obs;
    int32_t *rewards;
    uint8_t *dones;
    int32_t *land;
    int64_t *army_tot;
    int32_t *next_actions;        // fused actor output (nullptr: no actor)
    uint64_t actor_seed, step_idx;
};

struct SampleArgs {
    Geom g;
    uint64_t env_base, actor_seed, step_idx;
    const EnvScalars *sc;
    const int8_t *owner;
    const uint8_t *type;
    const int32_t *army;
    int32_t *actions;
};

uint32_t lds_bytes(const Geom &g);
hipError_t launch_step(const EnvArgs &a, int n_envs, hipStream_t stream);
hipError_t launch_reset(const EnvArgs &a, int n_envs, hipStream_t stream);
hipError_t launch_observe(const EnvArgs &a, int n_envs, hipStream_t stream);
hipError_t launch_sample(const SampleArgs &a, int n_envs, hipStream_t stream);

}  // namespace gen
