"""MI355X-native particle-filter resampling (arXiv 1202.6163, Murray 2012).

The computation lives in libresample.so (hand-written HIP for gfx950 behind
the C ABI of include/resample.h). ``paper_1202_6163_amd.api`` binds it with
the same function names; its names are re-exported here on first access, so
importing the package alone (e.g. for ``workloads``) needs no GPU library.
"""

_API_NAMES = ("resample_metropolis", "resample_metropolis_adaptive", "resample_stratified", "resample_systematic",
              "resample_multinomial", "resample_sorted", "resample_and_copy", "ancestors_to_offspring", "permute_copy", "rs_log_sum_exp", "rs_workspace_log_sum_exp",
              "metropolis_B", "rs_log_u_table", "rs_metropolis_set_tuning", "rs_metropolis_get_tuning",
              "workspace", "workspace_bytes", "RESAMPLERS")


def __getattr__(name):
    if name in _API_NAMES:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
