"""MI355X-native hot path of MH-DEOCT (arXiv 2311.06952): differential-evolution
fitness evaluation of classification trees on gfx950.

The computation lives in the HIP library ``libmhdeoct.so`` (C ABI in
``include/mhdeoct.h``); :mod:`paper_2311_06952_amd.capi` is its thin ctypes
binding, with torch used only for device memory and streams.
:mod:`paper_2311_06952_amd.synth` generates seeded synthetic inputs.
"""
from .capi import (Context, Dataset, MhError, Server, TileSet, autotune, cart, dataset,  # noqa
                   de_init, de_params, de_step, default_context, fitness_eval, load_library,
                   mh_train, predict, rank_encode, server_footprint, split1, subtree_solve,
                   tree_decode, tree_encode, tree_thresholds)

__all__ = ["Context", "Dataset", "MhError", "Server", "TileSet", "autotune", "cart", "dataset",
           "de_init",
           "de_params", "de_step", "default_context", "fitness_eval", "load_library", "mh_train",
           "predict", "rank_encode", "server_footprint", "split1", "subtree_solve", "tree_decode",
           "tree_encode", "tree_thresholds"]
