"""Plain FP64 CPU oracle for the layered-media Helmholtz sum.

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and by
the cpu_baseline leg of bench.py, never by the product path.  It shares no code
with the GPU library.
"""
