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

struct PoolArgs {
    GenParamsDev prm;            // common settings; cities and spawn distance per env
    uint64_t seed, env_base, actor_seed;
    uint32_t n_envs, wpg, lds_per_wave;
    const PoolDesc *desc;
    const uint32_t *order;       // work list: env of each slot
    EnvScalars *sc;
    int8_t *owner;
    uint8_t *type;
    int32_t *army;
    int32_t *actions;            // ragged int32, read and (with the actor) rewritten
    int32_t *rewards;
    uint8_t *dones;
    uint8_t *obs;
};

uint32_t lds_bytes(const Geom &g);
uint32_t lds_bytes_for(int S, int P);
int obs_variant(int HW, int P);
hipError_t launch_pool(const PoolArgs &a, int kind, bool act, uint32_t grid, hipStream_t stream);
hipError_t launch_step(const EnvArgs &a, int n_envs, hipStream_t stream);
hipError_t launch_reset(const EnvArgs &a, int n_envs, hipStream_t stream);
hipError_t launch_observe(const EnvArgs &a, int n_envs, hipStream_t stream);
hipError_t launch_sample(const SampleArgs &a, int n_envs, hipStream_t stream);

}  // namespace gen
