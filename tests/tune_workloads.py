"""Workloads the tuner test hands to its child processes (module:function form)."""
from paper_1608_06915_amd import synth


def small_channel():
    return synth.channel3d(32, 20, 16, 4, nu0=0.01)
