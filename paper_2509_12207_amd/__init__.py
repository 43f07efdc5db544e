"""Urgency-gated launching of deadline-bound GPU task chains on MI355X.

``capi`` binds the C-ABI of ``libug.so`` (include/ug.h); ``synth`` describes
seeded synthetic workloads; ``runner`` drives a workload through the gate on
torch-allocated device memory; ``build`` compiles the library with hipcc.
"""
