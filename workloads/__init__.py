"""Seeded synthetic inputs (scenes, poses, range images) shared by the tests,
the benchmark and the smoke check.  Holds no arithmetic of the method."""
from . import scenes, configs  # noqa: F401
