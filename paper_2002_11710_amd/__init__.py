"""MI355X-native Tabu search for air-ambulance fleet scheduling.

A thin ctypes binding over libatabu.so (include/atabu.h).  It only marshals
arguments: device buffers are torch CUDA tensors, streams are torch streams,
and every step of the method runs in the library's HIP kernels.  Importing
works without a GPU; calling anything that launches work needs the built
library and a gfx950 device, and fails loudly otherwise.
"""
from ._capi import (  # noqa: F401
    AT_EAGAIN, AT_EDEVICE, AT_EINFEAS, AT_EINVAL, AT_ENOMEM, AT_ERANGE, AT_NS, AT_OK, AT_TABU,
    FORM_BEST, FORM_SWEEP, SCHED_AUTO, SCHED_GLOBAL, SCHED_MULTI, SCHED_WAVE, SCHED_WG, AtError,
    DeviceInstance, Server,
    build_travel, build_travel_device, debug_eval_moves, lib, lib_path, solve, solve_batch,
    BatchResult, shutdown, solve_batch_flat, solve_noalloc, symbols, workspace_size,
)

__all__ = [
    "AT_OK", "AT_EINVAL", "AT_ERANGE", "AT_ENOMEM", "AT_EAGAIN", "AT_EDEVICE", "AT_EINFEAS",
    "AT_TABU", "AT_NS", "FORM_BEST", "FORM_SWEEP", "SCHED_AUTO", "SCHED_WG", "SCHED_MULTI",
    "SCHED_GLOBAL", "SCHED_WAVE", "AtError", "BatchResult", "solve_batch_flat",
    "DeviceInstance", "Server", "build_travel", "build_travel_device", "debug_eval_moves",
    "lib", "lib_path", "shutdown", "solve", "solve_batch", "solve_noalloc", "symbols",
    "workspace_size",
]
