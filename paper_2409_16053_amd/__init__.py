"""MI355X-native 3D Newtonian adiabatic hydro update on MeshBlocks.

The hot path (ghost-zone fill, cons-to-prim, PLM/PPM4 reconstruction -- and
PPMX or WENO-Z --, HLLC fluxes in x/y/z, flux divergence with a low-storage
SSP-RK stage update (RK1 to the ten-stage RK4), optional first-order flux
correction, CFL time-step reduction, and on statically refined meshes the
ghost slabs and flux correction at the level change) runs in hand-written HIP
kernels for gfx950 inside ``libhy.so``, reached through the C ABI declared in
``include/hy.h``. ``hy`` is the thin ctypes binding; ``problems`` builds
seeded synthetic initial conditions; ``serve`` is the continuous-batching
request loop.
"""
