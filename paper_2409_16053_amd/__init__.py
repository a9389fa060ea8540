"""MI355X-native 3D Newtonian adiabatic hydro update on MeshBlocks.

The hot path (ghost-zone fill, cons-to-prim, PLM/PPM4 reconstruction, HLLC
fluxes in x/y/z, flux divergence with an SSP-RK2 stage update, CFL time-step
reduction) runs in hand-written HIP kernels for gfx950 inside ``libhy.so``,
reached through the C ABI declared in ``include/hy.h``. ``hy`` is the thin
ctypes binding; ``problems`` builds seeded synthetic initial conditions.
"""
