"""MI355X-native loss-and-gradient library for gradient-trained NEP potentials."""
