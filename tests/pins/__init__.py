"""Independent closed forms and second routes that pin the CPU oracle.

Nothing here imports the oracle or the GPU package: each module restates a
textbook result (or the paper's own parametrization) in its own code.
"""
