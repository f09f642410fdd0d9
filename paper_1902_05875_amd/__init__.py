"""MI355X-native Taylor-expansion FMM for the 3-D Helmholtz sum in layered media."""
