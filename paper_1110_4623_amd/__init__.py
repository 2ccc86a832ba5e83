"""Inter-workgroup synchronization primitives for AMD Instinct MI355X (gfx950).

An MI355X-native implementation of the barriers, mutexes and semaphores of Stuart &
Owens, "Efficient Synchronization Primitives for GPUs" (2011), with the memory-system
microbenchmarks that classify a GPU (Sections 3-4), condition variables and queue
mutexes (the paper's future work and design alternatives), a persistent serving queue
built on the primitives, HIP-graph recording and an autotuner for their parameters.  The
compute path is libsp.so (hand-written HIP for gfx950, C ABI in include/sp.h); this
package is its binding.
"""

from ._native import SpError, SpNotResident, SpTimeout
from .api import (Barrier, Context, DeviceBuffer, Graph, Mutex, Semaphore,
                  barrier_hash_launches, bench_atomic, bench_fence, bounded_buffer, copy, litmus,
                  make_params, paper12, pingpong, serve, serve_launch_per_request,
                  shader_clock_mhz, stream_read)

__all__ = [
    "Barrier", "Context", "DeviceBuffer", "Graph", "Mutex", "Semaphore", "SpError",
    "SpNotResident", "SpTimeout", "barrier_hash_launches", "bench_atomic", "bench_fence",
    "bounded_buffer",
    "copy", "litmus", "make_params", "paper12", "pingpong", "serve",
    "serve_launch_per_request", "shader_clock_mhz", "stream_read",
]
