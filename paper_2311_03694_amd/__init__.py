"""MI355X (gfx950) implementation of the online stage of a Galerkin ROM whose advection
tensor is dense (G-ROM) or CP-decomposed (CPD-ROM), arXiv 2311.03694.

The compute path is librom.so (HIP kernels behind the C ABI of include/rom.h); this
package holds its sources (csrc/), its build script and a thin ctypes binding.
"""
from .binding import (  # noqa: F401
    DTYPES, EXPORTS, LIB_PATH, NonFinite, Rom, RomError, RomState, lib, rom_create, rom_destroy,
    rom_energy, rom_last_error, rom_nonlinear, rom_nonlinear_noalloc, rom_nonlinear_timed, rom_query, rom_set_tile, rom_state_create,
    rom_state_destroy, rom_state_get, rom_state_set, rom_state_set_slot, rom_state_u, rom_step, rom_step_async,
    rom_step_multi, rom_step_prepare, rom_step_sync, rom_tile_count, rom_cp_skew_layout, rom_cp_als, rom_cp_als_skew,
)
