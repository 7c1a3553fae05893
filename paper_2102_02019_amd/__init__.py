"""MI355X (gfx950) implementation of the LABFM hot path: stencil search,
Hermite-ABF weight construction, operator application and the isothermal
Navier-Stokes Runge-Kutta stages, behind the C ABI of include/labfm.h.

The HIP binding is imported lazily (``from paper_2102_02019_amd import labfm``)
so that the input generators can be used without a GPU."""

__all__ = ["inputs", "labfm"]
