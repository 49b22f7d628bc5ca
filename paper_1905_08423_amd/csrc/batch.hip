// Batched numeric launches (filled in below).
