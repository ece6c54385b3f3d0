"""MI355X-native flat-layer inversion of the 3D multi-frequency scalar
Helmholtz coefficient problem (Bakushinsky & Leonov, Algorithm 2)."""
