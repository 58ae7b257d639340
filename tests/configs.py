"""Launch configurations of the GPU parity tests: the library default and
the autotuner's stored pick for a workload (the configuration the benchmark
times)."""
from __future__ import annotations


def tuned_params(g, pl):
    from paper_2505_05643_amd import autotune
    sig = autotune.signature(g.n, pl.wh)
    params = autotune.cached_params(sig)
    assert params is not None, f"no autotune pick stored for {sig}"
    return params


def launch_configs(R, g, pl):
    """[(name, Params)]: the default and the tuned configuration."""
    return [("default", R.Params()), ("tuned", tuned_params(g, pl))]
