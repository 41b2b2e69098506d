"""pm4g: directly-follows graph discovery over columnar event logs on MI355X.

The compute path is the HIP library ``libpm4g.so`` behind the C ABI declared in
``include/pm4g.h``; :mod:`paper_2204_04898_amd.pm4g` is its thin binding.
Importing this package does not load the library.
"""
