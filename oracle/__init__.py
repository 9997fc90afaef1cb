"""Float64 reference of the Kino-PAX+ iteration -- test infrastructure only.

Used by tests/, the smoke check and the CPU-baseline leg of bench.py; the
planner package never imports it.
"""
