// hf_runtime.hpp -- internal declarations shared by the host translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/hfuse.h"
#include "hf_kernels.hpp"

namespace hf {

struct Slot {
  void* ptr = nullptr;
  size_t bytes = 0;
};

struct DeviceState {
  int device = 0;
  int num_cus = 0;
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;  // timing
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;   // two-stream baseline
  hipStream_t side = nullptr;                        // second stream if the caller gives none
  std::vector<Slot> slots;                           // scratch arena, one slot per concurrent task
  void* scrub = nullptr;                             // 1 GiB cache scrub buffer
  void* warm = nullptr;                              // sink of the warm-up kernel
  void* static_scratch = nullptr;                    // device address of the static scratch array
};

// Solo launches a featurisation made and their summed time (the learned
// tuner's profiling cost besides the candidates it profiles).
struct FeatCost {
  int launches = 0;
  double ms = 0.0;
};

int record_hip(hipError_t e);
DeviceState* device_state(int* status);
const KernelEntry* find_kernel(int ka, int kb, int block, int cap);
bool cap_in_menu(int cap);
int check_block(int block);
int validate_task(const hf_task* t);
int validate_fused(const hf_pair* pr, const hf_config* cfg);
int64_t scratch_bytes(const hf_task* t);
int prepare(const hf_task* t, void* scratch, DevTask* dt);
int arena_slot(DeviceState* s, int i, size_t bytes, void** out);
int launch_solo(DeviceState* s, const hf_task* t, int block, int grid, int slot, hipStream_t st);
int launch_fused(DeviceState* s, const hf_pair* pr, const hf_config* cfg, hipStream_t st, int* grid_used);
int launch_unfused(DeviceState* s, const hf_pair* pr, int block_a, int block_b, int mode,
                   hipStream_t s0, hipStream_t s1);
int wait_event(hipEvent_t ev);
int kernel_info(DeviceState* s, const void* fn, int block, hf_kernel_info* out);
void mlp_free();
int64_t useful_wgs(const hf_task* t, const DevTask& d, int waves);
int occupancy_grid(DeviceState* s, const void* fn, int block, int* wg_per_cu);

}  // namespace hf
