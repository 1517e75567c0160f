"""MI355X (gfx950) pipelined BiCGSafe solvers (Huynh & Suito, arXiv 2108.10591).

``pipesafe`` is the binding of the HIP library; ``workloads`` holds the seeded
synthetic inputs.  Importing the package loads neither.
"""
__version__ = "0.1.0"
