"""MI355X partitioned vector index: adaptive partition scanning on gfx950.

The compute path is the HIP library libquake_mi355x.so (C ABI in
include/quake.h); ``quake`` is its Python binding.
"""

from .quake import (  # noqa: F401
    Index,
    QuakeError,
    Server,
    load_library,
    quake_access_stats,
    quake_add_level,
    quake_adjust_levels,
    quake_autotune,
    quake_build,
    quake_candidates,
    quake_cap_table,
    quake_delete,
    quake_describe,
    quake_export,
    quake_export_top,
    quake_free,
    quake_insert,
    quake_insert_attrs,
    quake_load,
    quake_maintain,
    quake_profile,
    quake_profile_latency,
    quake_remove_level,
    quake_save,
    quake_search,
    quake_search_noalloc,
    quake_server_create,
    quake_server_delete,
    quake_server_destroy,
    quake_server_insert,
    quake_server_search,
    quake_server_stats,
    quake_server_wait,
    quake_set_tuning,
    quake_stats,
)
