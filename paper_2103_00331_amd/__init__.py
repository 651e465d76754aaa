"""cpmdp on MI355X: CP/Kronecker-structured Bellman backups in HIP for gfx950.

The GPU library (``csrc/`` -> ``libcpmdp.so``) is reached through the thin
ctypes binding in ``paper_2103_00331_amd.binding``; importing this package does
not load it, so the instance generator can be used on machines without a GPU.
"""

__all__ = ["instances", "binding"]
