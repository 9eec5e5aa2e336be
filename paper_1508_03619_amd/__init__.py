"""MI355X-native direction-optimizing BFS (GAP benchmark BFS kernel).

The compute path is the C-ABI library ``libgapbfs.so`` (hand-written HIP for
gfx950, declared in ``include/gapbfs.h``).  ``paper_1508_03619_amd.gapbfs``
is a thin ctypes binding with the same names; importing this package does not
load the library until a call needs it.
"""
from .gapbfs import (GapError, Graph, bc, bfs, bfs_batch, build_csr, free, graph_info, load,  # noqa: F401
                     library_path, set_params, get_params, library_defaults, last_stats, sssp,
                     SSSP_UNREACHABLE, cc, stream_status, bfs_noalloc, NOALLOC_SCRATCH_BYTES, shutdown,
                     Server, SERVE_RING,
                     device_query, stream_copy,
                     GAP_OK, GAP_EINVAL, GAP_ENOMEM, GAP_EDEVICE, GAP_EBUSY, GAP_EINTERNAL, GAP_ETIMEOUT)
