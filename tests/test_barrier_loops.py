"""The compiled kernels have no barrier inside a loop driven by the exec mask
(static check of hipcc's AMDGCN output; no GPU needed)."""
import os

from paper_1312_0138_amd import check_barriers


def test_every_barrier_loop_is_uniform(tmp_path):
    asm = check_barriers.device_asm(str(tmp_path / "kernels.s"))
    text = open(asm).read()
    report = check_barriers.check_text(text)
    assert any("k_slice" in k for k in report) and any("k_batch_run" in k for k in report)
    assert check_barriers.divergent_barrier_loops(text) == {}


def test_checker_flags_a_divergent_barrier_loop(tmp_path):
    """A loop whose exit depends on a value read from LDS, with single-lane
    regions at both ends of its body -- the shape that deadlocked a workgroup --
    must be reported."""
    src = tmp_path / "bad.hip"
    src.write_text(r'''
#include <hip/hip_runtime.h>
__global__ __launch_bounds__(256) void k_bad(unsigned* counter, unsigned total, unsigned* out) {
  __shared__ unsigned s[1];
  for (;;) {
    if (threadIdx.x == 0) s[0] = atomicAdd(counter, 1u);
    __syncthreads();
    const unsigned it = s[0];
    __syncthreads();
    if (it >= total) break;
    out[it * 256 + threadIdx.x] = it;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(counter + 1, it);
  }
}
''')
    asm = check_barriers.device_asm(str(tmp_path / "bad.s"), src=str(src))
    bad = check_barriers.divergent_barrier_loops(open(asm).read())
    assert any("k_bad" in k for k in bad)
