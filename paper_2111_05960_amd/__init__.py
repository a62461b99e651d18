"""MI355X-native coupled phi / c lattice-Boltzmann step of the grand-potential
phase-field model of dissolution and precipitation (arXiv:2111.05960).

The computation lives in libgplbm.so (HIP, gfx950) behind the C ABI of
include/gplbm.h; ``binding`` marshals arguments to it.
"""
from .binding import (Simulation, GplbmError, load, make_params,  # noqa: F401
                      gplbm_state_bytes, gplbm_checkpoint_bytes, gplbm_create,
                      gplbm_set_stream, gplbm_init_fields, gplbm_step, gplbm_step_count,
                      gplbm_read_fields, gplbm_diagnostics, gplbm_save_state,
                      gplbm_load_state, gplbm_schedule, gplbm_last_error, gplbm_destroy)
from .units import lattice_steps, to_lattice_units  # noqa: F401
