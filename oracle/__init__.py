"""FP64 oracle for the electromagnetic lattice Boltzmann hot path.

TEST INFRASTRUCTURE ONLY.  Importable by tests/, by the smoke check in
__graft_entry__.py and by the CPU-baseline leg of bench.py; the product
package (paper_2510_11042_amd) never imports it and shares no code with it.

Modules
  core      -- ctypes wrapper of lbm_oracle.c (literal 42-scalar scheme)
  analytic  -- Fresnel coefficients, lattice dispersion closed form
  mie       -- Lorenz-Mie series for circular cylinders and spheres
  ntff      -- near-to-far-field transform of DFT phasors -> |S|^2
"""
