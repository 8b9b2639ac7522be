"""MI355X-native asynchronous DG (ADG-AT) stepper: HIP kernels behind a C ABI."""
