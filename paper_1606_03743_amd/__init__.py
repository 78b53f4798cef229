"""MI355X (gfx950) library for the potential and field of charged BEM triangles and
rectangles by Gaussian cubature (Glueck & Hilk, arXiv:1606.03743).

    from paper_1606_03743_amd.bemc import Context

The HIP library is loaded lazily by ``bemc.load_library()``; importing the package does
not touch the GPU.  ``workloads`` builds seeded synthetic inputs.
"""
__all__ = ["bemc", "workloads"]
