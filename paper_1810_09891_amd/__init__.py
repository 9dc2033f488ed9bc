"""MI355X-native NFFT (placeholder: the HIP binding is added with the library)."""
