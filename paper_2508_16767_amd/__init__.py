"""MI355X-native Walk-on-Interfaces: HIP kernels for gfx950 behind the C ABI of include/woi.h."""
