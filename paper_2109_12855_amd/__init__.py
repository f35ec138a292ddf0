"""MI355X-native spike delivery (arXiv 2109.12855 hot path).

Importing the package loads nothing; ``paper_2109_12855_amd.sdeliver`` binds
the C ABI of ``libsdeliver.so`` and ``paper_2109_12855_amd.workloads`` holds
workload parameters and seeded input generators.
"""
