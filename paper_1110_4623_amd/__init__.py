"""Inter-workgroup synchronization primitives for AMD Instinct MI355X (gfx950).

An MI355X-native implementation of the barriers, mutexes and semaphores of Stuart &
Owens, "Efficient Synchronization Primitives for GPUs" (2011), with the memory-system
microbenchmarks that classify a GPU (Sections 3-4), a persistent serving queue built on
the primitives, and an autotuner for their parameters.  The compute path is libsp.so
(hand-written HIP for gfx950, C ABI in include/sp.h); this package is its binding.
"""

from .api import (Barrier, Context, DeviceBuffer, Graph, Mutex, Semaphore, barrier_hash_launches,
                  bounded_buffer,
                  bench_atomic, copy, litmus, make_params, paper12, pingpong, serve,
                  serve_launch_per_request, stream_read)
from ._native import SpError, SpNotResident, SpTimeout

__all__ = ["Barrier", "Context", "DeviceBuffer", "Graph", "Mutex", "Semaphore", "barrier_hash_launches",
           "bounded_buffer",
           "bench_atomic", "copy", "litmus", "make_params", "paper12", "pingpong", "serve",
           "serve_launch_per_request", "stream_read", "SpError",
           "SpNotResident", "SpTimeout"]
