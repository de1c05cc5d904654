"""MI355X-native dual proximal solvers (MINFBE, NAMA) for scenario-tree
stochastic optimal control (arXiv 2107.01745).

The compute path is the HIP library ``libstotree.so`` behind the C ABI of
``include/stotree.h``; ``paper_2107_01745_amd.stotree`` is its ctypes binding.
Importing this package loads nothing; the binding loads the library on first
use and raises if it has not been built.
"""
