"""Plain CPU oracle for the masked-Laplace inpainting path.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import anything from this package; the
product library never calls it and shares no code with it.

Everything is float64 and follows the paper's definitions directly:
  inpaint.py  -- the inpainting system (Sec. 2.1, eq. inp-discrete-lsi)
  tonal.py    -- tonal optimisation (Sec. 5, eqs. tonal-opt-minimisation and
                 tonal-normal-equations)
  densify.py  -- one Delaunay/Voronoi densification step (Sec. 4.1, Alg. 1)
  spatial.py  -- the Laplacian-dithered initial mask and the densification
                 loop around it (Sec. 4.2, Alg. 1)
  tonal_init.py -- Voronoi initialisation of tonal optimisation: Richardson
                 steps on cell-averaged interpolation constraints (Sec. 5.3)
"""
