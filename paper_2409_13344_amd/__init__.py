"""MI355X-native APPGA reconstruction for smoothed higher-order isotropic-TV PET.

Submodules are imported lazily: ``synth`` (seeded synthetic inputs) needs only
numpy; ``appga`` loads the HIP library ``libappga.so`` built for gfx950.
"""
