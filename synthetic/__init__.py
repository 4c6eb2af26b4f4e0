"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only draws random numbers and builds camera poses: it holds none
of the optimizer's or the renderer's arithmetic, so both the CPU oracle and the
HIP path can consume its outputs without sharing any computation.
"""
from .scenes import (  # noqa: F401
    Camera,
    SceneInputs,
    fibonacci_sphere,
    look_at,
    make_camera,
    n_params,
    config1_scene,
    config2_scene,
    config3_scene,
    config4_scene,
    serving_requests,
    request_scene,
    random_scene,
    tiny_scene,
)
