"""m-Cubes VEGAS sampling on AMD Instinct MI355X (gfx950).

The compiled library (``libmcubes.so``) is loaded on first use by
``paper_2202_01753_amd.mcubes``; importing the package itself loads nothing.
"""
