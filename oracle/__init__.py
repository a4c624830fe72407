"""FP64 CPU oracle of the MHDuet right-hand side (test infrastructure only).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use it.
"""
