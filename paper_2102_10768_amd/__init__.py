"""CST-based subgraph matching on AMD MI355X (gfx950).

The matching path (graph residency and label index, CST construction,
partition to the LDS budget, enumeration) is the HIP library ``libcstm.so``
behind the C ABI in ``include/cstm.h``; :mod:`paper_2102_10768_amd.cstm` is
its ctypes binding.
"""

from .cstm import (  # noqa: F401
    CST,
    Context,
    CstmError,
    Graph,
    batch_count,
    load_library,
)

__all__ = ["CST", "Context", "CstmError", "Graph", "batch_count", "load_library"]
